// Register-resident k x k triangular kernels for k <= 256 (FP64): Cholesky
// followed by the inverse of its factor, and the inverse of a given
// triangular matrix.  They serve the Cholesky-QR of C and R^T behind the
// stable CUR formula (the Remark on a stable CUR, eq. cur_stable) and the
// triangular inverses of the ID coefficients (Sec. 4, Z from L' of eq.
// def_LUPP).
//
// Layout: one 1024-thread workgroup per matrix; thread (tr, tc) = (tid % 32,
// tid / 32) holds S(tr + 32 a, tc + 32 b) for the lower blocks b <= a < NB
// (NB = ceil(k / 32)), i.e. the lower triangle lives block-cyclically in the
// register file of one CU (36 doubles per thread at k = 256).  Each step is a
// rank-1 update with one column (and one row) broadcast through LDS and one
// workgroup barrier; the vector for the next step is finished first and
// published into the other half of a double buffer, so its latency hides
// behind the bulk of the current update.
//
// Cholesky (right-looking): at step j every entry (i, c) with c > j takes
// S(i, c) -= L(i, j) L(c, j); column j + 1 is then final and is scaled by
// 1 / sqrt(S(j+1, j+1)) (hardware reciprocal square root refined by two
// Newton steps).
//
// Inverse of a lower triangular L (in place, Gauss-Jordan by columns): at
// step p, with x = row p of the partial inverse scaled by 1 / L(p, p),
// S(i, c) -= L(i, p) x(c) for i > p, c < p; S(i, p) = -L(i, p) / L(p, p);
// S(p, p) = 1 / L(p, p).  After the last step S holds L^{-1}.  An upper
// triangular input U is inverted as the lower matrix U^T and written back
// transposed.
#include "rpid_internal.hpp"

namespace rpid {
namespace {

constexpr int SW_MAXK = 256;

struct SweepJob {
  int k;             // order (<= 32 NB; padded with an identity block)
  const double* in;  // k x k input (lower part read, or upper part read transposed)
  int64_t ldi;
  const double* sub; // nullable: the lower part of sub is subtracted from the input
  int64_t lds;
  int in_upper;      // 1: input is upper triangular (read transposed)
  double* out;       // k x k output (full matrix written)
  int64_t ldo;
  int out_upper;     // 1: write the result transposed (upper triangular)
  double* fac;       // Cholesky only, nullable: R = L^T written here (full matrix)
  int64_t ldf;
  int64_t* status;   // Cholesky only: status_add + j + 1 if column j is not positive
  int status_add;
  int status_ok;     // 1: write 0 to *status on success
};

struct SweepArgs {
  int chol;  // 1: Cholesky of the (symmetric) input, then invert the factor
  int unit;  // inverse only: unit diagonal, the diagonal is not read
  SweepJob job[2];
};

__device__ __forceinline__ double sw_readlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// 1 / sqrt(d): hardware estimate and two Newton steps
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Shared state of one workgroup's sweep.
struct SweepLds {
  double colbuf[2][SW_MAXK];
  double rowbuf[2][SW_MAXK];
  double rd[SW_MAXK];  // 1 / diagonal of the triangular factor
  int fail;
};

// Thread grid 32 x TC: thread (tr, tc) = (tid % 32, tid / 32) holds rows
// tr + 32 a (row block a < NB) and columns tc + TC b (column block b); block
// (a, b) is stored when it meets the lower triangle, b <= bmax(a).
template <int TC>
struct Grid {
  static constexpr int NT = 32 * TC;
  static constexpr int bmax(int a) { return (32 * a + 31) / TC; }
  static constexpr int amin(int b) { return (TC * b) / 32; }
};

// Cholesky step j (0 <= j < k - 1); column j + 1 lies in column block B1.
// Same loop shape as the inverse step: the column-side factors L(c, j) stay
// in registers, the row-side factor L(i, j) is read from LDS per row block.
template <int TC, int NB, int NC, int B1>
__device__ __forceinline__ void chol_step(double (&v)[NB][NC], SweepLds& L, int j, int tr, int tc,
                                          int wave, int64_t* status, int status_add) {
  using G = Grid<TC>;
  constexpr int A0 = G::amin(B1);
  const double* pc = L.colbuf[j & 1];
  double cc[NC];
#pragma unroll
  for (int b = B1; b < NC; ++b) cc[b] = pc[tc + TC * b];
  if (tc + TC * B1 <= j) cc[B1] = 0.0;  // columns <= j are final
  // (1) column block B1 (holds column j + 1)
#pragma unroll
  for (int a = A0; a < NB; ++a) v[a][B1] = fma(-pc[tr + 32 * a], cc[B1], v[a][B1]);
  // (2) column j + 1 is final: scale it by 1 / sqrt of its diagonal, publish it
  const int town = (j + 1) % TC;
  if (wave == (town * 32) / 64) {
    double dsel = 0.0;
    const int ad = (j + 1) >> 5;
#pragma unroll
    for (int a = A0; a < NB; ++a)
      if (a == ad) dsel = v[a][B1];
    const double d = sw_readlane(dsel, (town * 32) % 64 + ((j + 1) & 31));
    if (tc == town) {
      const double y = rsqrt_nr(d);
#pragma unroll
      for (int a = A0; a < NB; ++a) {
        const int i = tr + 32 * a;
        const double l = (i > j + 1) ? v[a][B1] * y : (i == j + 1 ? d * y : 0.0);
        v[a][B1] = l;
        L.colbuf[(j + 1) & 1][i] = l;
      }
      if (tr == ((j + 1) & 31)) {
        L.rd[j + 1] = y;
        if (!(d > 0.0 && isfinite(d)) && !L.fail) {
          L.fail = 1;
          if (status) *status = status_add + j + 2;
        }
      }
    }
  }
  // (3) the remaining column blocks, row block by row block
#pragma unroll
  for (int a = A0; a < NB; ++a) {
    if constexpr (true) {
      const double cia = pc[tr + 32 * a];
#pragma unroll
      for (int b = B1 + 1; b < NC && b <= G::bmax(a); ++b) v[a][b] = fma(-cia, cc[b], v[a][b]);
    }
  }
  __syncthreads();
}

// The matrix is padded to 32 NB with an identity block, so every step below
// is valid and every trip count is a compile-time constant (no conditional
// step: a conditional step would keep two copies of the registers alive).
template <int TC, int NB, int NC, int JB>
__device__ __forceinline__ void chol_chunks(double (&v)[NB][NC], SweepLds& L, int tr, int tc,
                                            int wave, int64_t* status, int status_add) {
  if constexpr (JB < NC) {
#pragma unroll 1
    for (int j = TC * JB; j < TC * JB + TC - 1; ++j)
      chol_step<TC, NB, NC, JB>(v, L, j, tr, tc, wave, status, status_add);
    if constexpr (JB + 1 < NC) {
      // its column j + 1 starts column block JB + 1
      chol_step<TC, NB, NC, JB + 1>(v, L, TC * JB + TC - 1, tr, tc, wave, status, status_add);
    }
    chol_chunks<TC, NB, NC, JB + 1>(v, L, tr, tc, wave, status, status_add);
  }
}

// Inverse step p: column p in column block PB, row p + 1 in row block A1
// (A1 == NB: beyond the matrix), column p + 1 in column block QB.
template <int TC, int NB, int NC, int PB, int A1, int QB>
__device__ __forceinline__ void inv_step(double (&v)[NB][NC], SweepLds& L, int p, int tr,
                                         int tc) {
  using G = Grid<TC>;
  constexpr int A0 = G::amin(PB);  // row block of row p
  const double* pc = L.colbuf[p & 1];
  const double* pr = L.rowbuf[p & 1];
  const double dp = L.rd[p];
  double cc[NC];
#pragma unroll
  for (int b = 0; b <= PB; ++b) cc[b] = pr[tc + TC * b];
  // (1) row block A1 first: row p + 1 must be final before it is published
  if constexpr (A1 < NB) {
    const double cia = pc[tr + 32 * A1];
#pragma unroll
    for (int b = 0; b <= PB && b <= G::bmax(A1); ++b) v[A1][b] = fma(-cia, cc[b], v[A1][b]);
  }
  // (2) column p: S(i, p) = -L(i, p) / L(p, p) below, 1 / L(p, p) on the diagonal
  if (tc == p % TC) {
#pragma unroll
    for (int a = A0; a < NB; ++a) {
      const int i = tr + 32 * a;
      if (i > p) v[a][PB] = -v[a][PB] * dp;
      else if (i == p) v[a][PB] = dp;
    }
  }
  // (3) publish row p + 1 of the partial inverse, scaled, and column p + 1 of
  //     the original factor (zero on and above the diagonal)
  if constexpr (A1 < NB) {
    const int q = p + 1;
    {
      if (tr == (q & 31)) {
        const double dq = L.rd[q];
#pragma unroll
        for (int b = 0; b <= G::bmax(A1) && b < NC; ++b) {
          const int c = tc + TC * b;
          double x = 0.0;
          if (c < q) {
            x = v[A1][b] * dq;
            v[A1][b] = x;
          }
          L.rowbuf[q & 1][c] = x;
        }
      }
      if constexpr (QB < NC) {
        if (tc == q % TC) {
#pragma unroll
          for (int a = G::amin(QB); a < NB; ++a) {
            const int i = tr + 32 * a;
            L.colbuf[q & 1][i] = (i > q) ? v[a][QB] : 0.0;
          }
        }
      }
    }
  }
  // (4) the other row blocks
#pragma unroll
  for (int a = A0; a < NB; ++a) {
    if (a != A1) {
      const double cia = pc[tr + 32 * a];
#pragma unroll
      for (int b = 0; b <= PB && b <= G::bmax(a); ++b) v[a][b] = fma(-cia, cc[b], v[a][b]);
    }
  }
  __syncthreads();
}

template <int TC, int NB, int NC, int PB>
__device__ __forceinline__ void inv_chunks(double (&v)[NB][NC], SweepLds& L, int tr, int tc) {
  if constexpr (PB < NC) {
    constexpr int A1 = (TC * PB) / 32;        // row block of p + 1 inside the chunk
    constexpr int A1L = (TC * PB + TC) / 32;  // ... at its last step
#pragma unroll 1
    for (int p = TC * PB; p < TC * PB + TC - 1; ++p)
      inv_step<TC, NB, NC, PB, A1, PB>(v, L, p, tr, tc);
    inv_step<TC, NB, NC, PB, (A1L < NB ? A1L : NB), PB + 1>(v, L, TC * PB + TC - 1, tr, tc);
    inv_chunks<TC, NB, NC, PB + 1>(v, L, tr, tc);
  }
}

template <int TC, int NB>
__global__ __launch_bounds__(32 * TC) void sweep_kernel(SweepArgs args) {
  using G = Grid<TC>;
  constexpr int NC = (32 * NB) / TC;  // column blocks
  const SweepJob& job = args.job[blockIdx.x];
  const int k = job.k;
  const int tid = threadIdx.x;
  const int tr = tid & 31, tc = tid >> 5;
  const int wave = tid >> 6;

  __shared__ SweepLds L;
  for (int i = tid; i < 2 * SW_MAXK; i += G::NT) {
    (&L.colbuf[0][0])[i] = 0.0;
    (&L.rowbuf[0][0])[i] = 0.0;
  }
  if (tid == 0) L.fail = 0;

  // ---- load the lower triangle (padding rows/columns are zero) ------------
  const int64_t rs = job.in_upper ? job.ldi : 1, cs = job.in_upper ? 1 : job.ldi;
  double v[NB][NC];
#pragma unroll
  for (int a = 0; a < NB; ++a) {
#pragma unroll
    for (int b = 0; b <= G::bmax(a) && b < NC; ++b) {
      const int i = tr + 32 * a, c = tc + TC * b;
      // branch-free: clamped address, then select (identity padding beyond k)
      const bool inside = i < k && c < k && i >= c;
      const int ii = min(i, k - 1), cc2 = min(c, k - 1);
      const int64_t off = (int64_t)ii * rs + (int64_t)cc2 * cs;
      double x = job.in[off];
      if (job.sub) x -= job.sub[ii + (int64_t)cc2 * job.lds];
      v[a][b] = inside ? x : ((i == c) ? 1.0 : 0.0);
    }
  }
  __syncthreads();

  if (args.chol) {
    // ---- Cholesky: column 0 first (owners: tc == 0, wave 0 lanes 0..31) ---
    if (tc == 0) {
      const double d = sw_readlane(v[0][0], 0);
      const double y = rsqrt_nr(d);
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int i = tr + 32 * a;
        const double l = (i == 0) ? d * y : v[a][0] * y;
        v[a][0] = l;
        L.colbuf[0][i] = l;
      }
      if (tr == 0) {
        L.rd[0] = y;
        if (!(d > 0.0 && isfinite(d))) {
          L.fail = 1;
          if (job.status) *job.status = job.status_add + 1;
        }
      }
    }
    __syncthreads();
    // a breakdown only turns values into NaN: it is checked once at the end
    chol_chunks<TC, NB, NC, 0>(v, L, tr, tc, wave, job.status, job.status_add);
    if (L.fail) return;
    if (tid == 0 && job.status && job.status_ok) *job.status = 0;
    if (job.fac) {
#pragma unroll
      for (int a = 0; a < NB; ++a) {
#pragma unroll
        for (int b = 0; b <= G::bmax(a) && b < NC; ++b) {
          const int i = tr + 32 * a, c = tc + TC * b;
          if (i < k && c < k && i >= c) {
            job.fac[c + (int64_t)i * job.ldf] = v[a][b];
            if (i > c) job.fac[i + (int64_t)c * job.ldf] = 0.0;
          }
        }
      }
    }
    // reset the broadcast buffers for the inverse (the last step ended with
    // a barrier, so nobody reads them any more)
    for (int i = tid; i < 2 * SW_MAXK; i += G::NT) {
      (&L.colbuf[0][0])[i] = 0.0;
      (&L.rowbuf[0][0])[i] = 0.0;
    }
    __syncthreads();
  } else {
    // diagonal reciprocals of the given triangular matrix
#pragma unroll
    for (int a = 0; a < NB; ++a) {
#pragma unroll
      for (int b = 0; b <= G::bmax(a) && b < NC; ++b) {
        const int i = tr + 32 * a, c = tc + TC * b;
        if (i == c) L.rd[i] = (args.unit || i >= k) ? 1.0 : 1.0 / v[a][b];
      }
    }
    __syncthreads();
  }

  // ---- in-place inverse of the lower triangular S -------------------------
  // (column p of the factor is untouched until step p; row 0 of the partial
  // inverse has nothing left of the diagonal, so rowbuf[0] = 0 is its row)
  inv_chunks<TC, NB, NC, 0>(v, L, tr, tc);

  // ---- write the inverse (full matrix, zeros outside the triangle) --------
#pragma unroll
  for (int a = 0; a < NB; ++a) {
#pragma unroll
    for (int b = 0; b <= G::bmax(a) && b < NC; ++b) {
      const int i = tr + 32 * a, c = tc + TC * b;
      if (i < k && c < k && i >= c) {
        if (job.out_upper) {
          job.out[c + (int64_t)i * job.ldo] = v[a][b];
          if (i > c) job.out[i + (int64_t)c * job.ldo] = 0.0;
        } else {
          job.out[i + (int64_t)c * job.ldo] = v[a][b];
          if (i > c) job.out[c + (int64_t)i * job.ldo] = 0.0;
        }
      }
    }
  }
}

template <int TC, int NB>
int launch_sweep(rpid_ctx ctx, const SweepArgs& a, int batch) {
  hipLaunchKernelGGL((sweep_kernel<TC, NB>), dim3(batch), dim3(32 * TC), 0, ctx->stream, a);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int dispatch_sweep(rpid_ctx ctx, const SweepArgs& a, int batch) {
  int kmax = 0;
  for (int b = 0; b < batch; ++b) kmax = max(kmax, a.job[b].k);
  switch ((kmax + 31) / 32) {
    case 1: return launch_sweep<32, 1>(ctx, a, batch);
    case 2: return launch_sweep<32, 2>(ctx, a, batch);
    case 3: return launch_sweep<32, 3>(ctx, a, batch);
    case 4: return launch_sweep<32, 4>(ctx, a, batch);
    case 5: return launch_sweep<32, 5>(ctx, a, batch);
    default: return RPID_ERR_UNSUPPORTED;
  }
}

// Zero a rows x cols block of each of up to two matrices.
struct ZeroArgs {
  double* base[2];
  int64_t ld;
  int64_t rows, cols;
};

__global__ void zero_block_kernel(ZeroArgs z) {
  double* p = z.base[blockIdx.y];
  const int64_t total = z.rows * z.cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    p[(e % z.rows) + (e / z.rows) * z.ld] = 0.0;
}

int zero_blocks(rpid_ctx ctx, int batch, double* b0, double* b1, int64_t ld, int64_t rows,
                int64_t cols) {
  ZeroArgs z{{b0, b1}, ld, rows, cols};
  int64_t blocks = (rows * cols + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(zero_block_kernel, dim3((unsigned)blocks, (unsigned)batch), dim3(256), 0,
                     ctx->stream, z);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

SweepJob make_job(int k, const double* in, int64_t ldi, int in_upper, double* out, int64_t ldo,
                  int out_upper) {
  SweepJob j{};
  j.k = k;
  j.in = in;
  j.ldi = ldi;
  j.sub = nullptr;
  j.lds = 0;
  j.in_upper = in_upper;
  j.out = out;
  j.ldo = ldo;
  j.out_upper = out_upper;
  j.fac = nullptr;
  j.ldf = 0;
  j.status = nullptr;
  j.status_add = 0;
  j.status_ok = 0;
  return j;
}

// One launch holds a matrix of order <= 160 in registers; up to 288 the
// matrix is split once into 2 x 2 blocks (leading block 128); up to 512 the
// leading block of 128 is split off and the trailing block, of order k - 128,
// is treated the same way (recursively).
constexpr int64_t SW_ONE = 160;
constexpr int64_t SW_SPLIT = 128;
constexpr int64_t SW_MAX = 512;

// Cholesky G = R^T R and Winv = R^{-1} (upper) for one SPD matrix of any
// order up to SW_MAX by repeated splitting:
//   R11^T R11 = G11 (one sweep, W11 = R11^{-1}), R12 = W11^T G12,
//   S = G22 - R12^T R12 formed explicitly, R22 and W22 from S (the same
//   function), W12 = -W11 R12 W22, W21 = 0.
// A non-positive pivot at global column c writes c + 1 to *status (c counts
// from the first column of the outermost call: status_add); *status = 0 is
// written on success only by the outermost call (write_ok).
int chol_inverse_split(rpid_ctx ctx, int64_t k, const double* G, int64_t ldg, double* Winv,
                       int64_t ldw, int64_t* status, int status_add, bool write_ok,
                       size_t ws_tmp) {
  SweepArgs a{};
  a.chol = 1;
  a.unit = 0;
  const int64_t k1 = k <= SW_ONE ? k : SW_SPLIT, k2 = k - k1;
  a.job[0] = make_job((int)k1, G, ldg, 0, Winv, ldw, 1);
  a.job[0].status = status;
  a.job[0].status_add = status_add;
  a.job[0].status_ok = write_ok ? 1 : 0;
  RPID_CHECK(dispatch_sweep(ctx, a, 1));
  if (k2 == 0) return RPID_OK;
  Carve cv;
  cv.off = ws_tmp;
  const size_t o_R12 = cv.take<double>((size_t)k1 * k2);
  const size_t o_S = cv.take<double>((size_t)k2 * k2);
  const size_t o_T = cv.take<double>((size_t)k1 * k2);
  const size_t ws_next = cv.off;
  RPID_CHECK(ws_check(ctx, cv.off));
  double* R12 = ws_ptr<double>(ctx, o_R12);
  double* S = ws_ptr<double>(ctx, o_S);
  double* T = ws_ptr<double>(ctx, o_T);
  double* W22 = Winv + k1 + k1 * ldw;
  RPID_CHECK(dgemm(ctx, true, false, k1, k2, k1, 1.0, Winv, ldw, G + k1 * ldg, ldg, 0.0, R12, k1,
                   ws_next));
  RPID_CHECK(convert_matrix<double, double>(ctx, k2, k2, G + k1 + k1 * ldg, ldg, S, k2));
  RPID_CHECK(dgemm(ctx, true, false, k2, k2, k1, -1.0, R12, k1, R12, k1, 1.0, S, k2, ws_next));
  RPID_CHECK(chol_inverse_split(ctx, k2, S, k2, W22, ldw, status, status_add + (int)k1, false,
                                ws_next));
  RPID_CHECK(dgemm(ctx, false, false, k1, k2, k2, 1.0, R12, k1, W22, ldw, 0.0, T, k1, ws_next));
  RPID_CHECK(dgemm(ctx, false, false, k1, k2, k1, -1.0, Winv, ldw, T, k1, 0.0, Winv + k1 * ldw, ldw,
                   ws_next));
  return zero_blocks(ctx, 1, Winv + k1, nullptr, ldw, k2, k1);
}

}  // namespace

bool sweep_supported(int64_t k) { return k >= 1 && k <= SW_MAX; }

size_t sweep_scratch_bytes(int64_t k) {
  // R12, P, T for two matrices, then room for the GEMM partial sums
  return (size_t)6 * k * k * sizeof(double) + 256;
}

int chol_inverse_batched(rpid_ctx ctx, int batch, int64_t k, const double* G, int64_t ldg,
                         int64_t stride, double* Winv, int64_t ldw, int64_t wstride,
                         int64_t* status_dev, size_t ws_tmp) {
  if (!sweep_supported(k) || batch < 1 || batch > 2) return RPID_ERR_UNSUPPORTED;
  if (k > SW_SPLIT + SW_ONE) {
    if (batch != 1) return RPID_ERR_UNSUPPORTED;
    return chol_inverse_split(ctx, k, G, ldg, Winv, ldw, status_dev, 0, true, ws_tmp);
  }
  SweepArgs a{};
  a.chol = 1;
  a.unit = 0;
  if (k <= SW_ONE) {
    for (int b = 0; b < batch; ++b) {
      a.job[b] = make_job((int)k, G + b * stride, ldg, 0, Winv + b * wstride, ldw, 1);
      a.job[b].status = status_dev + b;
      a.job[b].status_ok = 1;
    }
    return dispatch_sweep(ctx, a, batch);
  }
  // G = [G11 G12; G12^T G22] = R^T R with R = [R11 R12; 0 R22]:
  //   R11^T R11 = G11, R12 = R11^{-T} G12, R22^T R22 = G22 - R12^T R12,
  //   R^{-1} = [W11, -W11 R12 W22; 0, W22] with W = inverses of the blocks.
  const int64_t k1 = SW_SPLIT, k2 = k - SW_SPLIT;
  Carve cv;
  cv.off = ws_tmp;
  const size_t o_R12 = cv.take<double>((size_t)2 * k1 * k2);
  const size_t o_P = cv.take<double>((size_t)2 * k2 * k2);
  const size_t o_T = cv.take<double>((size_t)2 * k1 * k2);
  const size_t ws_dg = cv.off;
  RPID_CHECK(ws_check(ctx, cv.off));
  for (int b = 0; b < batch; ++b) {
    a.job[b] = make_job((int)k1, G + b * stride, ldg, 0, Winv + b * wstride, ldw, 1);
    a.job[b].status = status_dev + b;
    a.job[b].status_ok = 1;
  }
  RPID_CHECK(dispatch_sweep(ctx, a, batch));
  for (int b = 0; b < batch; ++b) {
    const double* Gb = G + b * stride;
    double* Wb = Winv + b * wstride;
    double* R12 = ws_ptr<double>(ctx, o_R12) + b * k1 * k2;
    double* P = ws_ptr<double>(ctx, o_P) + b * k2 * k2;
    RPID_CHECK(dgemm(ctx, true, false, k1, k2, k1, 1.0, Wb, ldw, Gb + k1 * ldg, ldg, 0.0, R12, k1,
                     ws_dg));
    RPID_CHECK(dgemm(ctx, true, false, k2, k2, k1, 1.0, R12, k1, R12, k1, 0.0, P, k2, ws_dg));
  }
  for (int b = 0; b < batch; ++b) {
    a.job[b] = make_job((int)k2, G + b * stride + k1 + k1 * ldg, ldg, 0,
                        Winv + b * wstride + k1 + k1 * ldw, ldw, 1);
    a.job[b].sub = ws_ptr<double>(ctx, o_P) + b * k2 * k2;
    a.job[b].lds = k2;
    a.job[b].status = status_dev + b;
    a.job[b].status_add = (int)k1;
    a.job[b].status_ok = 0;
  }
  RPID_CHECK(dispatch_sweep(ctx, a, batch));
  for (int b = 0; b < batch; ++b) {
    double* Wb = Winv + b * wstride;
    double* R12 = ws_ptr<double>(ctx, o_R12) + b * k1 * k2;
    double* T = ws_ptr<double>(ctx, o_T) + b * k1 * k2;
    RPID_CHECK(dgemm(ctx, false, false, k1, k2, k2, 1.0, R12, k1, Wb + k1 + k1 * ldw, ldw, 0.0, T,
                     k1, ws_dg));
    RPID_CHECK(dgemm(ctx, false, false, k1, k2, k1, -1.0, Wb, ldw, T, k1, 0.0, Wb + k1 * ldw, ldw,
                     ws_dg));
  }
  return zero_blocks(ctx, batch, Winv + k1, batch > 1 ? Winv + wstride + k1 : nullptr, ldw, k2,
                     k1);
}

int tri_inverse_sweep(rpid_ctx ctx, int64_t k, const double* T, int64_t ldt, bool lower, bool unit,
                      double* W, int64_t ldw, size_t ws_tmp) {
  if (!sweep_supported(k)) return RPID_ERR_UNSUPPORTED;
  SweepArgs a{};
  a.chol = 0;
  a.unit = unit ? 1 : 0;
  const int up = lower ? 0 : 1;
  if (k <= SW_ONE) {
    a.job[0] = make_job((int)k, T, ldt, up, W, ldw, up);
    return dispatch_sweep(ctx, a, 1);
  }
  // both diagonal blocks (in one launch while the trailing one fits a
  // sweep; above that the trailing block by this function), then the
  // off-diagonal block:
  //   lower: W21 = -W22 T21 W11;  upper: W12 = -W11 T12 W22
  const int64_t k1 = SW_SPLIT, k2 = k - SW_SPLIT;
  Carve cv;
  cv.off = ws_tmp;
  const size_t o_Y = cv.take<double>((size_t)k1 * k2);
  const size_t ws_dg = cv.off;
  RPID_CHECK(ws_check(ctx, cv.off));
  double* Y = ws_ptr<double>(ctx, o_Y);
  a.job[0] = make_job((int)k1, T, ldt, up, W, ldw, up);
  if (k2 <= SW_ONE) {
    a.job[1] = make_job((int)k2, T + k1 + k1 * ldt, ldt, up, W + k1 + k1 * ldw, ldw, up);
    RPID_CHECK(dispatch_sweep(ctx, a, 2));
  } else {
    RPID_CHECK(dispatch_sweep(ctx, a, 1));
    RPID_CHECK(tri_inverse_sweep(ctx, k2, T + k1 + k1 * ldt, ldt, lower, unit, W + k1 + k1 * ldw, ldw,
                                 ws_dg));
  }
  const double* W11 = W;
  const double* W22 = W + k1 + k1 * ldw;
  if (lower) {
    RPID_CHECK(dgemm(ctx, false, false, k2, k1, k1, 1.0, T + k1, ldt, W11, ldw, 0.0, Y, k2, ws_dg));
    RPID_CHECK(dgemm(ctx, false, false, k2, k1, k2, -1.0, W22, ldw, Y, k2, 0.0, W + k1, ldw, ws_dg));
    return zero_blocks(ctx, 1, W + k1 * ldw, nullptr, ldw, k1, k2);
  }
  RPID_CHECK(dgemm(ctx, false, false, k1, k2, k2, 1.0, T + k1 * ldt, ldt, W22, ldw, 0.0, Y, k1,
                   ws_dg));
  RPID_CHECK(dgemm(ctx, false, false, k1, k2, k1, -1.0, W11, ldw, Y, k1, 0.0, W + k1 * ldw, ldw,
                   ws_dg));
  return zero_blocks(ctx, 1, W + k1, nullptr, ldw, k2, k1);
}

}  // namespace rpid
