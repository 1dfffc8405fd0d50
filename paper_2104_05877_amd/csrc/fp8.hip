// FP8 (OCP E4M3) form of the row sketch X = Omega A (Alg. 2, step 2).
//
//   ea[j] = largest e with max_i |A(i, j)| * 2^e <= 448 (0 for a zero column)
//   eo    = largest e with max |Omega| * 2^e <= 448
//   A_q(:, j) = e4m3(A(:, j) * 2^ea[j]),  Om_q = e4m3(Omega * 2^eo)
//   X(:, j)   = (Om_q A_q)(:, j) * 2^-(eo + ea[j])
//
// e4m3 rounds to nearest, ties to the even code; the power-of-two scales keep
// every scaled value within +-448, so nothing saturates, and undoing them in
// X is exact.  The product runs on the FP8 MFMA (16 x 16 x 128, FP32
// accumulation) through the common sketch kernel.  Non-finite entries give
// NaN codes, hence a non-finite X that the LUPP reports.
#include "rpid_internal.hpp"

namespace rpid {

namespace {

constexpr float E4M3_MAX = 448.0f;

// RNE conversion of |x| <= 448 (or NaN) to its E4M3 code.
__device__ __forceinline__ uint32_t e4m3_code(float x) {
  const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  if (!(a == a)) return 0x7Fu | sign;
  uint32_t code;
  if (a < 0.015625f) {
    // below the smallest normal 2^-6: multiples of 2^-9 (code 8 is 2^-6 itself)
    code = (uint32_t)__builtin_rintf(a * 512.0f);
  } else {
    uint32_t b = __float_as_uint(a);
    b += 0x7FFFFu + ((b >> 20) & 1u);  // round the 23-bit mantissa to 3 bits, ties to even
    code = (b >> 20) - ((127u - 7u) << 3);
    if (code > 0x7Eu) code = 0x7Eu;
  }
  return code | sign;
}

// largest e with mx * 2^e <= 448 (mx > 0 finite); 0 otherwise
__device__ __forceinline__ int scale_exp(float mx) {
  if (!(mx > 0.0f) || !isfinite(mx)) return 0;
  int e = 8 - ilogbf(mx);
  while (ldexpf(mx, e) > E4M3_MAX) --e;
  while (ldexpf(mx, e + 1) <= E4M3_MAX) ++e;
  return e;
}

__device__ __forceinline__ float block_max(float v, float* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  float r = red[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fmaxf(r, red[i]);
  __syncthreads();
  return r;
}

// Four E4M3 codes packed little-endian into one word.  Where all four values
// lie within +-448 the hardware conversion (two values per instruction,
// round to nearest even; it agrees with e4m3_code on every float of that
// range, checked on the device) forms them; otherwise (NaN, or a column whose
// scale was left at 1 because it holds a non-finite entry) e4m3_code does.
__device__ __forceinline__ uint32_t e4m3_pack4(float a, float b, float c, float d) {
  if (fabsf(a) <= E4M3_MAX && fabsf(b) <= E4M3_MAX && fabsf(c) <= E4M3_MAX &&
      fabsf(d) <= E4M3_MAX) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
  }
  return (e4m3_code(a) & 0xffu) | ((e4m3_code(b) & 0xffu) << 8) | ((e4m3_code(c) & 0xffu) << 16) |
         ((e4m3_code(d) & 0xffu) << 24);
}

__device__ __forceinline__ float scaled_or_nan(float v, int e) {
  return isfinite(v) ? ldexpf(v, e) : NAN;
}

// one workgroup per column: max |A(:, j)| -> ea[j], then the quantised column.
// Columns of up to 4 QC_NT QC_G rows are held in registers (128 values per
// thread, one workgroup per CU), so A is read once; longer columns take two
// passes.
constexpr int QC_NT = 512;
constexpr int QC_G = 32;

// Round-to-nearest-even to at most 3 significant mantissa bits reads only
// the sign, the exponent, the top 4 mantissa bits and whether any lower bit
// is set (E4M3 normals keep 3 bits, its subnormals fewer).  keep5 keeps
// those bits of a float, the last one in bit 18 (the top 4 bits rounded to
// odd at 5): the result rounds to the same code as the float at every
// power-of-two scale that keeps FP32 subnormal inputs away from the nonzero
// codes (scale exponents up to 116), infinities stay infinite and NaN stays
// NaN.  Two such floats share one register: one in bits 18..31, the other
// shifted down into bits 0..13.
__device__ __forceinline__ uint32_t keep5(uint32_t b) {
  return (b | ((b & 0x3FFFFu) + 0x3FFFFu)) & 0xFFFC0000u;
}

__device__ __forceinline__ uint32_t block_max_u32(uint32_t v, uint32_t* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  uint32_t r = red[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = max(r, red[i]);
  __syncthreads();
  return r;
}

// Columns of whole groups of 4 QC_NT rows (at most 4 QC_NT QC_G), 16-byte
// aligned: the same quantisation with one 16-byte load per group and thread,
// QC_WIN of them in flight at a time, and the column kept as keep5 fields,
// two to a register (64 registers per thread instead of 128), so that two
// workgroups share a CU and one's loads overlap the other's reduction and
// stores.  The largest |A(i, j)| comes from an integer maximum of the bit
// patterns without sign, which also tells a non-finite entry (the patterns
// from 0x7F800000 up).  A column with a non-finite entry, or scaled by more
// than 2^116 (largest entry below about 2^-108), is quantised again from A
// itself.
constexpr int QC_WIN = 12;
constexpr int QC_BUF_WORD3 = 0x00020000;  // raw 32-bit loads, out-of-range reads give 0
constexpr int QC_KEEP5_MAX_EXP = 116;

__global__ __launch_bounds__(QC_NT) __attribute__((amdgpu_waves_per_eu(4)))
void quantize_cols_v4_kernel(const float* A, int64_t m, int64_t lda, uint8_t* Aq, int64_t ldq, int* ea) {
  __shared__ uint32_t red[QC_NT / 64];
  const int64_t j = blockIdx.x;
  const int64_t t = threadIdx.x;
  const int ng = (int)(m / (4 * QC_NT));
  const float* col = A + j * lda;
  // buffer loads over the column's m rows: one offset register per thread,
  // the group's offset a scalar, and groups past the column read zeros
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(col), (short)0, (int)(4 * m), QC_BUF_WORD3);
  auto load = [&](int g) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(16 * t), 16 * QC_NT * g, 0);
    return make_uint4(v[0], v[1], v[2], v[3]);
  };
  uint4 q[QC_WIN];
#pragma unroll
  for (int g = 0; g < QC_WIN; ++g) q[g] = load(g);
  uint32_t h[QC_G][2];
  uint32_t mx = 0u;
#pragma unroll
  for (int g = 0; g < QC_G; ++g) {
    uint4 x = q[g % QC_WIN];
    if (g + QC_WIN < QC_G) q[g % QC_WIN] = load(g + QC_WIN);
    mx = max(mx, max(max(x.x & 0x7FFFFFFFu, x.y & 0x7FFFFFFFu), max(x.z & 0x7FFFFFFFu, x.w & 0x7FFFFFFFu)));
    h[g][0] = keep5(x.y) | (keep5(x.x) >> 18);
    h[g][1] = keep5(x.w) | (keep5(x.z) >> 18);
    // pin the packing here (an empty asm that reads and writes the pair):
    // sunk to the stores, it would keep the 128 loaded values alive instead
    asm volatile("" : "+v"(h[g][0]), "+v"(h[g][1]));
  }
  mx = block_max_u32(mx, red);
  const bool cnf_any = mx >= 0x7F800000u;
  const int ce = cnf_any ? 0 : scale_exp(__uint_as_float(mx));
  if (t == 0) ea[j] = ce;
  uint8_t* cq = Aq + j * ldq;
  if (!cnf_any && ce <= QC_KEEP5_MAX_EXP) {
    // every scaled value lies within +-448: the hardware conversion applies
#pragma unroll
    for (int g = 0; g < QC_G; ++g)
      if (g < ng) {
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(__uint_as_float(h[g][0] << 18), ce),
                                                ldexpf(__uint_as_float(h[g][0] & 0xFFFC0000u), ce), 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(__uint_as_float(h[g][1] << 18), ce),
                                            ldexpf(__uint_as_float(h[g][1] & 0xFFFC0000u), ce), w, true);
        *reinterpret_cast<int*>(cq + 4 * QC_NT * g + 4 * t) = w;
      }
  } else {
    // a non-finite entry (scale 1, NaN codes for NaN and infinities) or a
    // column of tiny values: quantise again from A itself
#pragma unroll 1
    for (int g = 0; g < ng; ++g) {
      const float4 x = *reinterpret_cast<const float4*>(col + 4 * QC_NT * g + 4 * t);
      *reinterpret_cast<uint32_t*>(cq + 4 * QC_NT * g + 4 * t) =
          e4m3_pack4(scaled_or_nan(x.x, ce), scaled_or_nan(x.y, ce), scaled_or_nan(x.z, ce), scaled_or_nan(x.w, ce));
    }
  }
}

__global__ __launch_bounds__(QC_NT) void quantize_cols_kernel(const float* A, int64_t m, int64_t lda,
                                                              uint8_t* Aq, int64_t ldq, int* ea) {
  __shared__ float red[QC_NT / 64];
  const int64_t j = blockIdx.x;
  const int64_t t = threadIdx.x;
  const float* col = A + j * lda;
  if (m <= (int64_t)QC_G * 4 * QC_NT) {
    // the whole column in registers (thread t holds elements 4 QC_NT g + 4 t + u),
    // read once, every load in flight together
    float v[QC_G][4];
#pragma unroll
    for (int g = 0; g < QC_G; ++g)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = 4 * QC_NT * g + 4 * t + u;
        v[g][u] = i < m ? col[i] : 0.0f;
      }
    float cm = 0.0f;
    bool cnf = false;
#pragma unroll
    for (int g = 0; g < QC_G; ++g)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float a = fabsf(v[g][u]);
        cnf |= !isfinite(a);
        cm = fmaxf(cm, a);
      }
    cm = block_max(cm, red);
    const bool cnf_any = __syncthreads_or(cnf);
    const int ce = cnf_any ? 0 : scale_exp(cm);
    if (t == 0) ea[j] = ce;
    uint8_t* cq = Aq + j * ldq;
#pragma unroll
    for (int g = 0; g < QC_G; ++g) {
      const int64_t i = 4 * QC_NT * g + 4 * t;
      const uint32_t w = e4m3_pack4(scaled_or_nan(v[g][0], ce), scaled_or_nan(v[g][1], ce),
                                    scaled_or_nan(v[g][2], ce), scaled_or_nan(v[g][3], ce));
      if (i + 3 < m) {  // ldq is a multiple of 512, so the 4-byte store is aligned
        *reinterpret_cast<uint32_t*>(cq + i) = w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i + u < m) cq[i + u] = (uint8_t)(w >> (8 * u));
      }
    }
    return;
  }
  // longer columns: two passes over the column, eight independent loads per
  // thread in flight per round
  float mx = 0.0f;
  bool nonfinite = false;
  for (int64_t b = 0; b < m; b += 8 * QC_NT) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = b + t + QC_NT * u;
      v[u] = i < m ? fabsf(col[i]) : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      nonfinite |= !isfinite(v[u]);
      mx = fmaxf(mx, v[u]);
    }
  }
  mx = block_max(mx, red);
  const bool any_nf = __syncthreads_or(nonfinite);
  const int e = any_nf ? 0 : scale_exp(mx);
  if (t == 0) ea[j] = e;
  // four codes per thread and one 4-byte store (ldq is a multiple of 512 and
  // the workspace regions are 256-byte aligned), bytes for the tail of m;
  // sixteen loads per thread in flight per round (four groups of four)
  uint8_t* q = Aq + j * ldq;
  const int64_t m4 = m & ~(int64_t)3;
  for (int64_t b = 0; b < m4; b += 16 * QC_NT) {
    float v[4][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = b + 4 * QC_NT * g + 4 * t + u;
        v[g][u] = i < m4 ? col[i] : 0.0f;
      }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int64_t i = b + 4 * QC_NT * g + 4 * t;
      if (i < m4) {  // i is a multiple of 4, so i + 3 < m4 as well
        *reinterpret_cast<uint32_t*>(q + i) =
            e4m3_pack4(scaled_or_nan(v[g][0], e), scaled_or_nan(v[g][1], e),
                       scaled_or_nan(v[g][2], e), scaled_or_nan(v[g][3], e));
      }
    }
  }
  for (int64_t i = m4 + t; i < m; i += QC_NT) {
    const float v = col[i];
    q[i] = (uint8_t)e4m3_code(isfinite(v) ? ldexpf(v, e) : NAN);
  }
}

// partial maxima of |Omega| (l x m), one per workgroup
__global__ __launch_bounds__(256) void omega_max_kernel(const float* Om, int64_t l, int64_t m,
                                                        int64_t ldo, float* part) {
  // each wave takes two columns per round, its lanes along the rows, so up
  // to sixteen loads per lane are in flight (no per-element index division)
  __shared__ float red[4];
  float mx = 0.0f;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < m; i += 2 * stride) {
    for (int64_t r0 = 0; r0 < l; r0 += 512) {
      float v[2][8];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t ic = i + c * stride, r = r0 + lane + 64 * u;
          v[c][u] = (ic < m && r < l) ? fabsf(Om[r + ic * ldo]) : 0.0f;
        }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int u = 0; u < 8; ++u) mx = (v[c][u] == v[c][u]) ? fmaxf(mx, v[c][u]) : INFINITY;
    }
  }
  mx = block_max(mx, red);
  if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

// the same partial maxima for a contiguous Omega (ldo == l): the l m values
// as one array, four per 16-byte load, four loads in flight per thread
__global__ __launch_bounds__(256) void omega_max_flat_kernel(const float* Om, int64_t total,
                                                             float* part) {
  __shared__ float red[4];
  float mx = 0.0f;
  auto take = [&](float x) {
    const float a = fabsf(x);
    mx = (a == a) ? fmaxf(mx, a) : INFINITY;
  };
  const int64_t n4 = total / 4;
  const float4* O4 = reinterpret_cast<const float4*>(Om);
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = O4[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      take(v[u].x);
      take(v[u].y);
      take(v[u].z);
      take(v[u].w);
    }
  }
  for (; i < n4; i += stride) {
    const float4 v = O4[i];
    take(v.x);
    take(v.y);
    take(v.z);
    take(v.w);
  }
  if (blockIdx.x == 0 && threadIdx.x < total - 4 * n4) take(Om[4 * n4 + threadIdx.x]);
  mx = block_max(mx, red);
  if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

// eo from the partial maxima (one workgroup)
__global__ __launch_bounds__(256) void omega_scale_kernel(const float* part, int nparts, int* eo) {
  __shared__ float red[4];
  float pm = 0.0f;
  for (int i = threadIdx.x; i < nparts; i += 256) pm = fmaxf(pm, part[i]);
  const int e = scale_exp(block_max(pm, red));
  if (threadIdx.x == 0) *eo = e;
}

// Pt_q = e4m3(Omega^T * 2^eo) (m x l, ldq) through 32 x 32 LDS tiles
__global__ __launch_bounds__(256) void quantize_omega_t_kernel(const float* Om, int64_t l, int64_t m,
                                                               int64_t ldo, const int* eo,
                                                               uint8_t* Ptq, int64_t ldq) {
  __shared__ float tile[32][33];
  const int e = *eo;
  const int64_t r0 = (int64_t)blockIdx.y * 32, i0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t r = r0 + tx, i = i0 + yy;
    tile[yy][tx] = (r < l && i < m) ? Om[r + i * ldo] : 0.0f;
  }
  __syncthreads();
  // each thread: four consecutive codes of one row of Pt_q, one 4-byte store
  // (ldq is a multiple of 512 and i0 of 32, so it is aligned)
  const int rr = threadIdx.x >> 3, c4 = (threadIdx.x & 7) * 4;
  const int64_t r = r0 + rr, i = i0 + c4;
  if (r < l && i < m) {
    const uint32_t w = e4m3_pack4(scaled_or_nan(tile[c4][rr], e), scaled_or_nan(tile[c4 + 1][rr], e),
                                  scaled_or_nan(tile[c4 + 2][rr], e), scaled_or_nan(tile[c4 + 3][rr], e));
    uint8_t* dst = Ptq + i + r * ldq;
    if (i + 3 < m) {
      *reinterpret_cast<uint32_t*>(dst) = w;
    } else {
      for (int u = 0; u < 4; ++u)
        if (i + u < m) dst[u] = (uint8_t)(w >> (8 * u));
    }
  }
}

// X(:, j) *= 2^-(eo + ea[j])
__global__ void unscale_kernel(float* X, int64_t l, int64_t n, int64_t ldx, const int* ea,
                               const int* eo) {
  const int64_t total = l * n;
  const int e0 = *eo;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % l, j = e / l;
    X[r + j * ldx] = ldexpf(X[r + j * ldx], -(e0 + ea[j]));
  }
}

constexpr int OMAX_PARTS = 4096;

}  // namespace

size_t sketch_fp8_workspace(int64_t m, int64_t n, int64_t l) {
  const int64_t mq = (m + 511) / 512 * 512;  // quantised rows padded to whole stage pairs
  return (size_t)mq * n + (size_t)mq * l + (size_t)n * sizeof(int) + 64 +
         OMAX_PARTS * sizeof(float) + 4096;
}

int sketch_fp8(rpid_ctx ctx, const float* A, int64_t m, int64_t n, int64_t lda, const float* Om,
               int64_t l, int64_t ldo, float* X, int64_t ldx, size_t ws_off) {
  // quantised copies padded with zero codes to a multiple of 512 rows, so the
  // streaming kernel (pairs of 256-deep stages, 16-byte aligned) applies
  const int64_t mq = (m + 511) / 512 * 512;
  Carve cv;
  cv.off = ws_off;
  const size_t o_Aq = cv.take<uint8_t>((size_t)mq * n);
  const size_t o_Pq = cv.take<uint8_t>((size_t)mq * l);
  const size_t o_ea = cv.take<int>((size_t)n);
  const size_t o_eo = cv.take<int>(16);
  const size_t o_part = cv.take<float>(OMAX_PARTS);
  const size_t o_gemm = cv.off;
  RPID_CHECK(ws_check(ctx, o_gemm));
  uint8_t* Aq = ws_ptr<uint8_t>(ctx, o_Aq);
  uint8_t* Pq = ws_ptr<uint8_t>(ctx, o_Pq);
  int* ea = ws_ptr<int>(ctx, o_ea);
  int* eo = ws_ptr<int>(ctx, o_eo);
  float* part = ws_ptr<float>(ctx, o_part);
  if (mq > m) {
    // zero codes in the padding rows of both operands (mq is a multiple of 512)
    RPID_CHECK(launch_fill_u64(ctx, reinterpret_cast<uint64_t*>(Aq), (size_t)mq * n / 8, 0ull));
    RPID_CHECK(launch_fill_u64(ctx, reinterpret_cast<uint64_t*>(Pq), (size_t)mq * l / 8, 0ull));
  }
  if (reinterpret_cast<uintptr_t>(A) % 16 == 0 && lda % 4 == 0 && m % (4 * QC_NT) == 0 &&
      m <= (int64_t)QC_G * 4 * QC_NT)
    hipLaunchKernelGGL(quantize_cols_v4_kernel, dim3((unsigned)n), dim3(QC_NT), 0, ctx->stream, A, m, lda,
                       Aq, mq, ea);
  else
    hipLaunchKernelGGL(quantize_cols_kernel, dim3((unsigned)n), dim3(QC_NT), 0, ctx->stream, A, m, lda,
                       Aq, mq, ea);
  RPID_HIP_CHECK(hipGetLastError());
  // at least eight columns of Omega per workgroup (two rounds of its four waves)
  const int parts = (int)std::min<int64_t>(OMAX_PARTS, (m + 7) / 8);
  if (ldo == l && reinterpret_cast<uintptr_t>(Om) % 16 == 0)
    hipLaunchKernelGGL(omega_max_flat_kernel, dim3(parts), dim3(256), 0, ctx->stream, Om, l * m, part);
  else
    hipLaunchKernelGGL(omega_max_kernel, dim3(parts), dim3(256), 0, ctx->stream, Om, l, m, ldo, part);
  RPID_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(omega_scale_kernel, dim3(1), dim3(256), 0, ctx->stream, part, parts, eo);
  RPID_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(quantize_omega_t_kernel, dim3((unsigned)((m + 31) / 32), (unsigned)((l + 31) / 32)),
                     dim3(256), 0, ctx->stream, Om, l, m, ldo, eo, Pq, mq);
  RPID_HIP_CHECK(hipGetLastError());
  RPID_CHECK(sketch_e4m3(ctx, Pq, mq, Aq, mq, mq, n, l, X, ldx, o_gemm));
  int64_t blocks = (l * n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(unscale_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, X, l, n, ldx,
                     ea, eo);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

}  // namespace rpid
