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

// Split a linear index into (i, j) of a rows x cols array; 32-bit division
// when the sizes allow (64-bit division is emulated and slow on the GPU).
__device__ __forceinline__ void split_index(int64_t e, int64_t rows, int64_t& i, int64_t& j) {
  if (e < 0x7fffffff && rows < 0x7fffffff) {
    const unsigned ue = (unsigned)e, ur = (unsigned)rows;
    i = ue % ur;
    j = ue / ur;
  } else {
    i = e % rows;
    j = e / rows;
  }
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
    int64_t i, j;
    split_index(e, rows, i, j);
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
    int64_t i, t;
    split_index(e, m, i, t);
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
    int64_t t, j;
    split_index(e, k, t, j);
    const int64_t i = I[t];
    R[t + j * ldr] =
        cvt_from_double<TD>((i >= 0 && i < nrows) ? load_as_double<TS>(A, i + j * lda) : 0.0);
  }
}

// Rt(j, t) = A(I[t], j): the rows A(I, :) written transposed (n x k), j
// fastest so the writes are contiguous; indices outside [0, nrows) give zeros.
template <typename TS>
__global__ void gather_rows_t_kernel(int64_t k, int64_t n, const TS* A, int64_t lda, int64_t nrows,
                                     const int64_t* I, double* Rt, int64_t ldr) {
  const int64_t total = k * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t j, t;
    split_index(e, n, j, t);
    const int64_t i = I[t];
    Rt[j + t * ldr] = (i >= 0 && i < nrows) ? load_as_double<TS>(A, i + j * lda) : 0.0;
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

// Z(:, J[t]) = e_t; entries of J outside [0, n) are skipped
__global__ void identity_cols_kernel(int64_t k, int64_t n, const int64_t* J, double* Z, int64_t ldz) {
  const int64_t total = k * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t c, t;
    split_index(e, k, c, t);
    const int64_t j = J[t];
    if (j >= 0 && j < n) Z[c + j * ldz] = (c == t) ? 1.0 : 0.0;
  }
}

__global__ void split_bf16_kernel(int64_t rows, int64_t cols, const double* S, int64_t lds,
                                  int parts, uint16_t* D, int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i, j;
    split_index(e, rows, i, j);
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
// takes NR right-hand sides; 256/NR threads share one right-hand side and
// split the dot products of each block of 16 unknowns, whose partial sums
// are combined in LDS before one thread does the 16 x 16 substitution.  The
// 16 rows of op(T) of the current block and the unknowns solved so far are
// kept in LDS (no dependent global loads in the inner loop).
// ---------------------------------------------------------------------------
constexpr int TB_ = 16;

template <typename TBt, int NR>
__global__ __launch_bounds__(256) void tri_solve_kernel(int64_t k, int64_t nrhs, const double* T,
                                                        int64_t ldt, bool trans, bool lower_op,
                                                        bool unit, const TBt* B, int64_t brs,
                                                        int64_t bcs, double* X, int64_t xrs,
                                                        int64_t xcs) {
  constexpr int PART = 256 / NR;
  constexpr int TPT = 2;  // op(T) columns staged per thread per block (k <= 512)
  extern __shared__ double sm[];
  const int64_t kx = k + 1;                // padded row of xs (avoids bank conflicts)
  double* blk = sm;                        // TB_ x k: blk[i * k + d] = op(T)(c0 + i, d)
  double* xs = sm + TB_ * k;               // NR x kx: right-hand sides, then unknowns
  double* part = xs + (int64_t)NR * kx;    // PART x NR x (TB_ + 1)
  const int tid = threadIdx.x;
  const int rl = tid % NR;  // right-hand side within the workgroup
  const int pt = tid / NR;  // partial-sum slot
  const int64_t r0 = (int64_t)blockIdx.x * NR;
  const int ki = (int)k;
  const int64_t nb = (k + TB_ - 1) / TB_;

  // prologue: every right-hand side of the workgroup into LDS (independent loads)
  for (int base = 0; base < NR * ki; base += 256 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + tid + 256 * u;
      const int c = idx / NR, q = idx % NR;
      v[u] = (idx < NR * ki && r0 + q < nrhs) ? load_as_double<TBt>(B, (r0 + q) * bcs + (int64_t)c * brs)
                                              : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + tid + 256 * u;
      if (idx < NR * ki) xs[(idx % NR) * kx + idx / NR] = v[u];
    }
  }
  // rows of op(T) for a block, prefetched into registers one block ahead
  double tv[TPT][TB_];
  auto fetchT = [&](int64_t blkid) {
    const int64_t c0 = blkid * TB_;
#pragma unroll
    for (int h = 0; h < TPT; ++h) {
      const int d = tid + 256 * h;
#pragma unroll
      for (int i = 0; i < TB_; ++i) {
        const int64_t row = c0 + i;
        tv[h][i] = (row < k && d < ki) ? (trans ? T[d + row * ldt] : T[row + (int64_t)d * ldt]) : 0.0;
      }
    }
  };
  fetchT(lower_op ? 0 : nb - 1);
  for (int64_t bb = 0; bb < nb; ++bb) {
    const int64_t blkid = lower_op ? bb : nb - 1 - bb;
    const int64_t c0 = blkid * TB_;
    const int bs = (int)min((int64_t)TB_, k - c0);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < TPT; ++h) {
      const int d = tid + 256 * h;
      if (d < ki) {
#pragma unroll
        for (int i = 0; i < TB_; ++i) blk[i * k + d] = tv[h][i];
      }
    }
    __syncthreads();
    if (bb + 1 < nb) fetchT(lower_op ? bb + 1 : nb - 2 - bb);
    // partial dot products with the unknowns already solved
    double acc[TB_];
#pragma unroll
    for (int i = 0; i < TB_; ++i) acc[i] = 0.0;
    const int64_t dlo = lower_op ? 0 : c0 + bs;
    const int64_t dhi = lower_op ? c0 : k;
    for (int64_t d = dlo + pt; d < dhi; d += PART) {
      const double xd = xs[rl * kx + d];
#pragma unroll
      for (int i = 0; i < TB_; ++i) acc[i] = fma(blk[i * k + d], xd, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < TB_; ++i) part[(pt * NR + rl) * (TB_ + 1) + i] = acc[i];
    __syncthreads();
    if (pt == 0) {
      double v[TB_];
#pragma unroll
      for (int i = 0; i < TB_; ++i) {
        double sum = 0.0;
#pragma unroll
        for (int p = 0; p < PART; ++p) sum += part[(p * NR + rl) * (TB_ + 1) + i];
        v[i] = (i < bs) ? xs[rl * kx + c0 + i] - sum : 0.0;
      }
      // column-oriented substitution: once unknown i2 is final, the updates
      // of the remaining unknowns are independent of each other
      if (lower_op) {
#pragma unroll
        for (int i2 = 0; i2 < TB_; ++i2) {
          if (i2 < bs) {
            if (!unit) v[i2] /= blk[i2 * k + c0 + i2];
#pragma unroll
            for (int i = i2 + 1; i < TB_; ++i) v[i] = fma(-blk[i * k + c0 + i2], v[i2], v[i]);
          }
        }
      } else {
#pragma unroll
        for (int i2 = TB_ - 1; i2 >= 0; --i2) {
          if (i2 < bs) {
            if (!unit) v[i2] /= blk[i2 * k + c0 + i2];
#pragma unroll
            for (int i = 0; i < i2; ++i) v[i] = fma(-blk[i * k + c0 + i2], v[i2], v[i]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < TB_; ++i)
        if (i < bs) xs[rl * kx + c0 + i] = v[i];
    }
  }
  __syncthreads();
  // epilogue: the unknowns to X
  for (int idx = tid; idx < NR * ki; idx += 256) {
    const int c = idx / NR, q = idx % NR;
    if (r0 + q < nrhs) X[(r0 + q) * xcs + (int64_t)c * xrs] = xs[q * kx + c];
  }
}

// ---------------------------------------------------------------------------
// Inverse of a k x k triangular matrix (k <= 512): W = T^{-1}, T lower or
// upper, unit or not.  One wave per column c of W: lane l holds rows
// l + 64 j of the column; column-oriented substitution (once unknown i is
// final it is broadcast with readlane and every lane updates its rows with
// column i of T); the diagonal reciprocals are computed once into LDS and the
// T columns are loaded ahead of their step.  No workgroup barrier inside the
// loop; all columns proceed in parallel.
// ---------------------------------------------------------------------------
constexpr int TI_MAXJ = 8;  // rows per lane (k <= 512)

template <int NJ, int D>
__global__ __launch_bounds__(256) void tri_inverse_kernel(int k, const double* T, int64_t ldt,
                                                          bool lower, bool unit, double* W,
                                                          int64_t ldw) {
  __shared__ double rdiag[512];
  const int tid = threadIdx.x, lane = tid & 63;
  for (int i = tid; i < k; i += blockDim.x) rdiag[i] = unit ? 1.0 : 1.0 / T[i + (int64_t)i * ldt];
  __syncthreads();
  const int c = blockIdx.x * 4 + (tid >> 6);
  if (c >= k) return;
  double x[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) x[j] = (lane + 64 * j == c) ? 1.0 : 0.0;
  // T(r, i) for this lane's rows r = lane + 64 j and column i (0 outside the
  // part of the column that updates unknowns after i)
  auto colT = [&](int i, double* out) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int r = lane + 64 * j;
      const bool need = (i >= 0 && i < k) && (lower ? (r > i && r < k) : (r < i));
      out[j] = need ? T[r + (int64_t)i * ldt] : 0.0;
    }
  };
  const int nsteps = lower ? k - c : c + 1;
  const int step = lower ? 1 : -1;
  // ring of D columns of T in flight
  double ring[D][NJ];
#pragma unroll
  for (int d = 0; d < D; ++d) colT(c + step * d, ring[d]);
  for (int s0 = 0; s0 < nsteps; s0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int sidx = s0 + d;
      if (sidx < nsteps) {
        const int i = c + step * sidx;
        const int jl = i >> 6, ll = i & 63;
        double xi = 0.0;
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          if (j == jl) xi = x[j];
        xi = __shfl(xi, ll, 64) * rdiag[i];
        double tc[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) tc[j] = ring[d][j];
        colT(c + step * (sidx + D), ring[d]);  // refill this slot D steps ahead
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          if (j == jl && lane == ll) x[j] = xi;
          x[j] = fma(-tc[j], xi, x[j]);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int r = lane + 64 * j;
    if (r < k) W[r + (int64_t)c * ldw] = x[j];
  }
}

// ---------------------------------------------------------------------------
// Cholesky G = L L^T of k x k SPD matrices (k <= 512), one 1024-thread
// workgroup per matrix, right-looking by panels of CB columns:
//  (a) the CB x CB diagonal block is factored by one wave in registers
//      (lane r holds row r; columns are broadcast with lane shuffles);
//  (b) every row below solves x L_D^T = G(row, panel) (one row per thread);
//  (c) the trailing lower triangle is updated with the panel held in LDS.
// The matrix stays in global memory (L2-resident); at the end R = L^T is
// written to the upper triangle and the strict lower triangle is zeroed.
// ---------------------------------------------------------------------------
constexpr int CB = 32;

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__global__ __launch_bounds__(1024) void cholesky_kernel(int64_t k, double* Gall, int64_t ldg,
                                                        int64_t stride, int64_t* status) {
  double* G = Gall + (int64_t)blockIdx.x * stride;
  extern __shared__ double pan[];  // k x (CB + 1) panel: pan[r * PS + c] = L(j0 + bs + r, j0 + c)
  constexpr int PS = CB + 1;       // padded row (avoids bank conflicts)
  __shared__ double dg[CB][CB + 1];
  __shared__ double rdg[CB];  // reciprocals of the diagonal of the current block
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int64_t j0 = 0; j0 < k; j0 += CB) {
    const int bs = (int)min((int64_t)CB, k - j0);
    // (a) diagonal block: wave 0 factors it with row `lane` in registers; the
    //     column of each step is broadcast through LDS (a wave's LDS accesses
    //     complete in program order, so no barrier is needed inside the loop)
    for (int e = tid; e < CB * CB; e += blockDim.x) {
      const int r = e / CB, c = e % CB;
      dg[r][c] = (r < bs && c < bs && c <= r) ? G[(j0 + r) + (j0 + c) * ldg] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      // cross-lane values are read from registers with readlane (uniform
      // lane index: c and c2 are constants of the unrolled loops)
      double a[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c) a[c] = (lane < CB) ? dg[lane][c] : 0.0;
      int fail = -1;
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        if (c < bs) {
          const double dcc = readlane_f64(a[c], c);
          if ((!(dcc > 0.0) || !isfinite(dcc)) && fail < 0) fail = c;
          // y ~ dcc^{-1/2}: hardware estimate refined by one Newton step
          double y = __builtin_amdgcn_rsq(dcc);
          y = y * fma(-0.5 * dcc * y, y, 1.5);
          if (lane == c) a[c] = dcc * y;
          if (lane > c) a[c] = a[c] * y;
          if (lane == c) rdg[c] = y;
#pragma unroll
          for (int c2 = c + 1; c2 < CB; ++c2) {
            if (c2 < bs) {
              const double l2 = readlane_f64(a[c], c2);
              if (lane >= c2) a[c2] = fma(-a[c], l2, a[c2]);
            }
          }
        }
      }
      if (lane < bs) {
#pragma unroll
        for (int c = 0; c < CB; ++c) dg[lane][c] = (c <= lane) ? a[c] : 0.0;
      }
      if (fail >= 0 && lane == 0) {
        bad = 1;
        status[blockIdx.x] = j0 + fail + 1;
      }
    }
    __syncthreads();
    if (bad) break;
    // write the factored diagonal block back (lower part)
    for (int e = tid; e < CB * CB; e += blockDim.x) {
      const int r = e / CB, c = e % CB;
      if (r < bs && c <= r) G[(j0 + r) + (j0 + c) * ldg] = dg[r][c];
    }
    // (b) rows below the block: x L_D^T = g  (forward substitution)
    const int64_t nb = k - j0 - bs;
    // (rows below exist only when bs == CB); each thread solves its row in
    // place in the LDS panel
    for (int64_t i = tid; i < nb; i += blockDim.x) {
      const int64_t row = j0 + bs + i;
      double* x = &pan[i * PS];
      double g[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c) g[c] = G[row + (j0 + c) * ldg];
#pragma unroll
      for (int c = 0; c < CB; ++c) x[c] = g[c];
      for (int c2 = 0; c2 < CB; ++c2) {
        const double xc = x[c2] * rdg[c2];
        x[c2] = xc;
        for (int c = c2 + 1; c < CB; ++c) x[c] = fma(-xc, dg[c][c2], x[c]);
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) G[row + (j0 + c) * ldg] = x[c];
    }
    __syncthreads();
    // (c) trailing update of the lower triangle, G(r, c) -= sum_p L(r, p) L(c, p):
    //     thread -> (row r, column group); its row of the panel sits in
    //     registers, the column's panel row is an LDS broadcast across the wave
    if (nb > 0) {
      const int nbi = (int)nb;
      const int groups = max(1, (int)blockDim.x / nbi);
      const int ri = tid % nbi, cg = tid / nbi;
      if (cg < groups) {
        double pr[CB];
#pragma unroll
        for (int p = 0; p < CB; ++p) pr[p] = pan[ri * PS + p];
        double* grow = G + (j0 + bs + ri);
        for (int c0 = cg; c0 <= ri; c0 += 4 * groups) {
          double v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int cc = c0 + u * groups;
            v[u] = (cc <= ri) ? grow[(j0 + bs + cc) * ldg] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int cc = c0 + u * groups;
            if (cc <= ri) {
              double acc = v[u];
#pragma unroll
              for (int p = 0; p < CB; ++p) acc = fma(-pr[p], pan[cc * PS + p], acc);
              grow[(j0 + bs + cc) * ldg] = acc;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (!bad) {
    if (tid == 0) status[blockIdx.x] = 0;
    const int ki = (int)k;
    for (int j = 0; j < ki; ++j)
      for (int i = tid; i < j; i += blockDim.x) G[i + j * ldg] = G[j + i * ldg];
    __syncthreads();
    for (int j = 0; j < ki; ++j)
      for (int i = j + 1 + tid; i < ki; i += blockDim.x) G[i + j * ldg] = 0.0;
  }
}

__global__ void axpy_kernel(int64_t rows, int64_t cols, double alpha, const double* S,
                            int64_t lds, double* D, int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i, j;
    split_index(e, rows, i, j);
    D[i + j * ldd] = fma(alpha, S[i + j * lds], D[i + j * ldd]);
  }
}

__global__ void zero_block_kernel(int64_t rows, int64_t cols, double* D, int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i, j;
    split_index(e, rows, i, j);
    D[i + j * ldd] = 0.0;
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

template <typename TS>
int gather_rows_t(rpid_ctx ctx, int64_t k, int64_t n, const TS* A, int64_t lda, int64_t nrows,
                  const int64_t* I, double* Rt, int64_t ldr) {
  hipLaunchKernelGGL((gather_rows_t_kernel<TS>), dim3(grid_for(k * n)), dim3(256), 0, ctx->stream, k, n, A,
                     lda, nrows, I, Rt, ldr);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}
template int gather_rows_t<double>(rpid_ctx, int64_t, int64_t, const double*, int64_t, int64_t,
                                   const int64_t*, double*, int64_t);
template int gather_rows_t<float>(rpid_ctx, int64_t, int64_t, const float*, int64_t, int64_t,
                                  const int64_t*, double*, int64_t);
template int gather_rows_t<uint16_t>(rpid_ctx, int64_t, int64_t, const uint16_t*, int64_t, int64_t,
                                     const int64_t*, double*, int64_t);

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

int set_identity_columns(rpid_ctx ctx, int64_t k, int64_t n, const int64_t* J, double* Z, int64_t ldz) {
  hipLaunchKernelGGL(identity_cols_kernel, dim3(grid_for(k * k)), dim3(256), 0, ctx->stream, k, n, J,
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

template <typename TBt, int NR>
static int tri_solve_nr(rpid_ctx ctx, int64_t k, int64_t nrhs, const double* T, int64_t ldt,
                        bool trans, bool lower_op, bool unit, const TBt* B, int64_t brs,
                        int64_t bcs, double* X, int64_t xrs, int64_t xcs) {
  const size_t shmem =
      sizeof(double) * ((size_t)TB_ * k + (size_t)NR * (k + 1) + (size_t)256 * (TB_ + 1));
  if (shmem > 160 * 1024) return RPID_ERR_UNSUPPORTED;
  const void* fn = reinterpret_cast<const void*>(tri_solve_kernel<TBt, NR>);
  RPID_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL((tri_solve_kernel<TBt, NR>), dim3((unsigned)((nrhs + NR - 1) / NR)),
                     dim3(256), shmem, ctx->stream, k, nrhs, T, ldt, trans, lower_op, unit, B,
                     brs, bcs, X, xrs, xcs);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

template <typename TBt>
int tri_solve(rpid_ctx ctx, int64_t k, int64_t nrhs, const double* T, int64_t ldt, bool trans,
              bool lower_op, bool unit, const TBt* B, int64_t brs, int64_t bcs, double* X,
              int64_t xrs, int64_t xcs) {
  if (nrhs <= 0 || k <= 0) return RPID_OK;
  // right-hand sides per workgroup: as many as the LDS holds (and enough
  // workgroups to spread over the chip)
  if (k <= 256 && nrhs >= 32 * 64) return tri_solve_nr<TBt, 32>(ctx, k, nrhs, T, ldt, trans, lower_op, unit, B, brs, bcs, X, xrs, xcs);
  if (k <= 512) return tri_solve_nr<TBt, 8>(ctx, k, nrhs, T, ldt, trans, lower_op, unit, B, brs, bcs, X, xrs, xcs);
  if (k <= 1024) return tri_solve_nr<TBt, 2>(ctx, k, nrhs, T, ldt, trans, lower_op, unit, B, brs, bcs, X, xrs, xcs);
  return RPID_ERR_UNSUPPORTED;
}

int tri_inverse(rpid_ctx ctx, int64_t k, const double* T, int64_t ldt, bool lower, bool unit,
                double* W, int64_t ldw, size_t ws_tmp) {
  if (k < 1) return RPID_OK;
  if (sweep_supported(k)) return tri_inverse_sweep(ctx, k, T, ldt, lower, unit, W, ldw, ws_tmp);
  if (k > 512 && k <= 1024) {
    // 2 x 2 blocks of orders h and k - h (both <= 512): the diagonal blocks of
    // W are the inverses of T's, the off-diagonal block is
    //   lower: W21 = -W22 (T21 W11),   upper: W12 = -W11 (T12 W22),
    // and the other off-diagonal block is zero.
    const int64_t h = k / 2, h2 = k - h;
    Carve cv;
    cv.off = ws_tmp;
    const size_t o_P = cv.take<double>((size_t)h * h2);
    const size_t o_rest = cv.off;
    RPID_CHECK(ws_check(ctx, o_rest));
    double* P = ws_ptr<double>(ctx, o_P);
    const double* T22 = T + h + h * ldt;
    double* W22 = W + h + h * ldw;
    RPID_CHECK(tri_inverse(ctx, h, T, ldt, lower, unit, W, ldw, o_rest));
    RPID_CHECK(tri_inverse(ctx, h2, T22, ldt, lower, unit, W22, ldw, o_rest));
    if (lower) {
      RPID_CHECK(dgemm(ctx, false, false, h2, h, h, 1.0, T + h, ldt, W, ldw, 0.0, P, h2, o_rest));
      RPID_CHECK(dgemm(ctx, false, false, h2, h, h2, -1.0, W22, ldw, P, h2, 0.0, W + h, ldw, o_rest));
      hipLaunchKernelGGL(zero_block_kernel, dim3(grid_for(h * h2)), dim3(256), 0, ctx->stream, h, h2,
                         W + h * ldw, ldw);
    } else {
      RPID_CHECK(dgemm(ctx, false, false, h, h2, h2, 1.0, T + h * ldt, ldt, W22, ldw, 0.0, P, h, o_rest));
      RPID_CHECK(dgemm(ctx, false, false, h, h2, h, -1.0, W, ldw, P, h, 0.0, W + h * ldw, ldw, o_rest));
      hipLaunchKernelGGL(zero_block_kernel, dim3(grid_for(h * h2)), dim3(256), 0, ctx->stream, h2, h,
                         W + h, ldw);
    }
    RPID_HIP_CHECK(hipGetLastError());
    return RPID_OK;
  }
  const unsigned blocks = (unsigned)((k + 3) / 4);
  if (k <= 256)
    hipLaunchKernelGGL((tri_inverse_kernel<4, 8>), dim3(blocks), dim3(256), 0, ctx->stream, (int)k, T,
                       ldt, lower, unit, W, ldw);
  else if (k <= 512)
    hipLaunchKernelGGL((tri_inverse_kernel<8, 4>), dim3(blocks), dim3(256), 0, ctx->stream, (int)k, T,
                       ldt, lower, unit, W, ldw);
  else
    return RPID_ERR_UNSUPPORTED;
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

int cholesky_batched(rpid_ctx ctx, int batch, int64_t k, double* G, int64_t ldg, int64_t stride,
                     int64_t* status_dev) {
  if (k > 512) return RPID_ERR_UNSUPPORTED;
  const size_t shmem = (size_t)k * (CB + 1) * sizeof(double);
  RPID_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(cholesky_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL(cholesky_kernel, dim3(batch), dim3(1024), shmem, ctx->stream, k, G, ldg,
                     stride, status_dev);
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
