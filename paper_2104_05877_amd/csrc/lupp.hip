// Tall-panel LU with partial pivoting (column-wise LUPP of eq. def_LUPP, as
// used by Alg. 2 steps 3 and 4), as one persistent cooperative kernel.
//
// Panel: n x k matrix P(i, j) = base[i * rs + j * cs] (i = candidate, j = step).
// Step t: pivot p_t = argmax over remaining i of |P^(t)(i, t)|, ties to the
// smallest i; multipliers P^(t)(i, t) / P^(t)(p_t, t); Schur update of
// columns t+1..k-1 of the remaining rows.
//
// Layout on the GPU:
//  * workgroup g owns rows [g R, g R + R); thread j (< k) owns column j of
//    those rows in R registers, so the panel lives in the register files of
//    the whole chip (8192 x 256 FP64 = 16 MB over 128 workgroups);
//  * the column of the current step is mirrored in LDS so that one wave
//    finds the workgroup's candidate with a 64-lane argmax;
//  * each step every workgroup publishes its candidate row into a slot and
//    the candidate's |value| into a per-step word (release, agent scope);
//    every workgroup polls the G words of the step (acquire), reduces them
//    identically (largest |value|, ties to the smallest workgroup, which owns
//    the smallest rows), reads the winning row, and updates its registers.
//  One device-wide exchange per pivot; no second kernel launch per step.
#include "rpid_internal.hpp"

#include <hip/hip_cooperative_groups.h>

namespace rpid {

static constexpr uint64_t kSentinel = ~0ull;
static constexpr unsigned kSpinLimit = 1u << 26;

template <typename T>
struct LuppArgs {
  const T* base;
  int64_t rs, cs;
  int64_t n;
  int k;
  int kpad;
  int64_t* J;
  T* Lf;
  int64_t ldl;
  T* Uf;
  int64_t ldu;
  T* diag;
  uint64_t* slot_val;  // k x G words: |candidate| bits of step t, workgroup g
  int64_t* slot_idx;   // 2 x G candidate row indices (double buffered)
  T* slot_row;         // 2 x G x kpad candidate rows (double buffered)
  unsigned* flags;     // [0] non-finite count, [1] abort
  int64_t* status;     // 0, t+1 (zero pivot), or a negative RPID_ERR code
};

template <typename T>
__device__ __forceinline__ uint64_t to_bits(T v);
template <>
__device__ __forceinline__ uint64_t to_bits<double>(double v) {
  return (uint64_t)__double_as_longlong(v);
}
template <>
__device__ __forceinline__ uint64_t to_bits<float>(float v) {
  return (uint64_t)__float_as_uint(v);
}
template <typename T>
__device__ __forceinline__ T from_bits(uint64_t b);
template <>
__device__ __forceinline__ double from_bits<double>(uint64_t b) {
  return __longlong_as_double((long long)b);
}
template <>
__device__ __forceinline__ float from_bits<float>(uint64_t b) {
  return __uint_as_float((unsigned)b);
}
template <>
__device__ __forceinline__ int64_t from_bits<int64_t>(uint64_t b) {
  return (int64_t)b;
}

template <typename T>
__device__ __forceinline__ T load_coherent(const T* p) {
  if constexpr (sizeof(T) == 8) {
    uint64_t b = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    return from_bits<T>(b);
  } else {
    unsigned b = __hip_atomic_load(reinterpret_cast<const unsigned*>(p), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    return from_bits<T>(b);
  }
}

// (value, index) argmax across a 64-lane wave: larger value wins, ties go to
// the smaller index.  Invalid entries carry value -2 (never a modulus).
template <typename T>
__device__ __forceinline__ void wave_argmax(T& v, int& i) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    T ov = __shfl_xor(v, off, 64);
    int oi = __shfl_xor(i, off, 64);
    bool take = (ov > v) || (ov == v && oi < i);
    v = take ? ov : v;
    i = take ? oi : i;
  }
}

template <typename T, int R, int NTMAX>
__global__ __launch_bounds__(NTMAX) void lupp_panel_kernel(LuppArgs<T> a) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int k = a.k;
  const int64_t row0 = (int64_t)g * R;
  const int lane = tid & 63;
  const int wid = tid >> 6;

  __shared__ T colbuf[R];      // column of the current step, this workgroup's rows
  __shared__ T mult[R];        // multipliers of the current step (0 for frozen rows)
  __shared__ int alive[R];     // 1 while the row has not been chosen as a pivot
  __shared__ T red_v[16];
  __shared__ int red_i[16];
  __shared__ int sh_bq;
  __shared__ T sh_best;
  __shared__ int sh_gw;
  __shared__ T sh_gbest;
  __shared__ int sh_stop;
  __shared__ int sh_nonfinite;

  // ---- load this workgroup's rows of the panel into registers ------------
  T s[R];
  bool bad = false;
  if (tid < k) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t row = row0 + q;
      T v = T(0);
      if (row < a.n) v = a.base[row * a.rs + (int64_t)tid * a.cs];
      bad |= !isfinite(v);
      s[q] = v;
    }
  }
  for (int q = tid; q < R; q += nt) alive[q] = (row0 + q < a.n) ? 1 : 0;
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < R; ++q) colbuf[q] = s[q];
  }
  if (__any(bad) && lane == 0) atomicAdd(&a.flags[0], 1u);
  __syncthreads();

  int t = 0;
  int64_t final_status = 0;
  for (; t < k; ++t) {
    const int par = t & 1;
    // ---- (1) candidate of this workgroup: one wave over the LDS column ----
    if (wid == 0) {
      T bv = T(-2);
      int bi = R;
      for (int q = lane; q < R; q += 64) {
        if (alive[q]) {
          T v = fabs(colbuf[q]);
          if (v > bv) {  // ascending q: strict > keeps the smallest index
            bv = v;
            bi = q;
          }
        }
      }
      wave_argmax(bv, bi);
      if (lane == 0) {
        sh_bq = bi;
        sh_best = bv;
        sh_stop = 0;
      }
    }
    __syncthreads();
    const int bq = sh_bq;

    // ---- (2) publish the candidate row and its |value| --------------------
    T* myrow = a.slot_row + ((size_t)par * G + g) * a.kpad;
    if (tid >= t && tid < k) {
      T v = T(0);
#pragma unroll
      for (int q = 0; q < R; ++q) v = (q == bq) ? s[q] : v;
      myrow[tid] = v;
    }
    if (tid == 0) a.slot_idx[par * G + g] = (bq < R) ? row0 + bq : -1;
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      const T pub = (bq < R) ? sh_best : T(-1);
      __hip_atomic_store(&a.slot_val[(size_t)t * G + g], to_bits<T>(pub), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    }

    // ---- (3) wait for every workgroup's word of step t, reduce ------------
    T cv = T(-2);
    int ci = 0x7fffffff;
    for (int i = tid; i < G; i += nt) {
      uint64_t b;
      unsigned spins = 0;
      while (true) {
        b = __hip_atomic_load(&a.slot_val[(size_t)t * G + i], __ATOMIC_ACQUIRE,
                              __HIP_MEMORY_SCOPE_AGENT);
        if (b != kSentinel) break;
        if ((++spins & 255u) == 0) {
          if (__hip_atomic_load(&a.flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
              spins > kSpinLimit) {
            __hip_atomic_store(&a.flags[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh_stop = 1;
            break;
          }
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (b != kSentinel) {
        const T v = from_bits<T>(b);
        if (v > cv || (v == cv && i < ci)) {
          cv = v;
          ci = i;
        }
      }
    }
    wave_argmax(cv, ci);
    if (lane == 0) {
      red_v[wid] = cv;
      red_i[wid] = ci;
    }
    __syncthreads();
    if (sh_stop) {
      final_status = RPID_ERR_TIMEOUT;
      break;
    }
    if (wid == 0) {
      const int nw = nt >> 6;
      T v = (lane < nw) ? red_v[lane] : T(-2);
      int i = (lane < nw) ? red_i[lane] : 0x7fffffff;
      wave_argmax(v, i);
      if (lane == 0) {
        sh_gw = i;
        sh_gbest = v;
        sh_nonfinite = (t == 0) ? (int)__hip_atomic_load(&a.flags[0], __ATOMIC_ACQUIRE,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                : 0;
      }
    }
    __syncthreads();
    if (sh_nonfinite != 0) {
      final_status = RPID_ERR_NONFINITE;
      break;
    }
    const int gw = sh_gw;
    const T gbest = sh_gbest;
    if (!(gbest > T(0))) {  // exactly zero pivot (or no candidate left)
      final_status = t + 1;
      break;
    }

    // ---- (4) read the pivot row, record outputs ----------------------------
    const T* wrow = a.slot_row + ((size_t)par * G + gw) * a.kpad;
    const int64_t prow = load_coherent(&a.slot_idx[par * G + gw]);
    const T pv = load_coherent(&wrow[t]);
    T uj = T(0);
    if (tid > t && tid < k) uj = load_coherent(&wrow[tid]);
    if (g == gw && tid == 0) alive[prow - row0] = 0;
    if (g == 0) {
      if (tid == 0) {
        a.J[t] = prow;
        if (a.diag) a.diag[t] = fabs(pv);
      }
      if (tid < k) a.Uf[t + (int64_t)tid * a.ldu] = (tid >= t) ? load_coherent(&wrow[tid]) : T(0);
    }
    __syncthreads();

    // ---- (5) multipliers (one per row, coalesced L writes) -----------------
    for (int q = tid; q < R; q += nt) {
      const int64_t row = row0 + q;
      const T mq = alive[q] ? colbuf[q] / pv : T(0);
      mult[q] = mq;
      if (row < a.n) a.Lf[row + (int64_t)t * a.ldl] = alive[q] ? mq : (row == prow ? T(1) : T(0));
    }
    __syncthreads();

    // ---- (6) Schur update of this workgroup's rows, columns t+1..k-1 -------
    if (tid > t && tid < k) {
#pragma unroll
      for (int q = 0; q < R; ++q) s[q] = fma(-mult[q], uj, s[q]);
      if (tid == t + 1) {
#pragma unroll
        for (int q = 0; q < R; ++q) colbuf[q] = s[q];
      }
    }
    __syncthreads();
  }
  if (g == 0 && tid == 0) *a.status = final_status;
}

size_t lupp_workspace_bytes(rpid_ctx ctx, int64_t n, int64_t k, int elem_bytes) {
  (void)ctx;
  const int64_t G = (n + 15) / 16;  // upper bound (smallest R)
  const int64_t kpad = (k + 63) / 64 * 64;
  size_t b = 0;
  b += (size_t)k * G * 8 + 256;
  b += (size_t)2 * G * 8 + 256;
  b += (size_t)2 * G * kpad * elem_bytes + 256;
  b += 256;
  return b;
}

__global__ void fill_u64_kernel(uint64_t* p, size_t count, uint64_t value) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = value;
}

int launch_fill_u64(rpid_ctx ctx, uint64_t* p, size_t count, uint64_t value) {
  if (count == 0) return RPID_OK;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, p, count,
                     value);
  RPID_HIP_CHECK(hipGetLastError());
  return RPID_OK;
}

// VGPRs a thread may spend on its R panel values: one wave per SIMD (256
// threads) or two (512) leave 256 registers per wave, four (1024) leave 128;
// the rest is kept for temporaries.
static constexpr int row_reg_budget(int ntmax) { return ntmax <= 512 ? 160 : 80; }

template <typename T, int R, int NTMAX>
static int launch_lupp_R(rpid_ctx ctx, LuppArgs<T> a, int G, int nt) {
  if constexpr (R * (int)sizeof(T) / 4 > row_reg_budget(NTMAX)) {
    return RPID_ERR_UNSUPPORTED;
  } else {
    void* kargs[] = {&a};
    const void* fn = reinterpret_cast<const void*>(lupp_panel_kernel<T, R, NTMAX>);
    int per_cu = 0;
    RPID_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, 0));
    if (per_cu < 1 || (int64_t)per_cu * ctx->num_cu < G) return RPID_ERR_LAUNCH;
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(nt), kargs, 0, ctx->stream);
    if (e != hipSuccess) return RPID_ERR_LAUNCH;
    return RPID_OK;
  }
}

// Largest rows-per-thread R whose register array fits row_reg_budget.
static int max_rows(int ntmax, int elem_bytes) {
  const int budget = row_reg_budget(ntmax);
  int r = 128;
  while (r > 16 && r * elem_bytes / 4 > budget) r /= 2;
  return r;
}

template <typename T, int NTMAX>
static int dispatch_R(rpid_ctx ctx, LuppArgs<T> a, int R, int G, int nt) {
  switch (R) {
    case 16: return launch_lupp_R<T, 16, NTMAX>(ctx, a, G, nt);
    case 32: return launch_lupp_R<T, 32, NTMAX>(ctx, a, G, nt);
    case 64: return launch_lupp_R<T, 64, NTMAX>(ctx, a, G, nt);
    case 128: return launch_lupp_R<T, 128, NTMAX>(ctx, a, G, nt);
    default: return RPID_ERR_UNSUPPORTED;
  }
}

template <typename T>
int lupp_panel(rpid_ctx ctx, const T* base, int64_t rs, int64_t cs, int64_t n, int64_t k,
               int64_t* J, T* Lf, int64_t ldl, T* Uf, int64_t ldu, T* diag, size_t ws_off,
               int64_t* status_dev) {
  if (k < 1 || k > 1024 || n < k) return RPID_ERR_UNSUPPORTED;
  const int nt = (int)((k + 63) / 64 * 64);
  const int ntmax = nt <= 256 ? 256 : (nt <= 512 ? 512 : 1024);
  // Rows per workgroup: the smallest R whose grid fits one workgroup per CU
  // (more rows per workgroup cost registers, fewer cost polling), capped by
  // the register budget.
  const int rmax = max_rows(ntmax, (int)sizeof(T));
  int R = rmax;
  for (int c = 16; c <= rmax; c *= 2) {
    if ((n + c - 1) / c <= ctx->num_cu) {
      R = c;
      break;
    }
  }
  const int64_t G64 = (n + R - 1) / R;
  if (G64 > 4096) return RPID_ERR_UNSUPPORTED;
  const int G = (int)G64;
  const int kpad = nt;

  Carve cv;
  cv.off = ws_off;
  size_t o_val = cv.take<uint64_t>((size_t)k * G);
  size_t o_idx = cv.take<int64_t>((size_t)2 * G);
  size_t o_row = cv.take<T>((size_t)2 * G * kpad);
  size_t o_flags = cv.take<uint64_t>(1);
  RPID_CHECK(ws_check(ctx, cv.off));

  LuppArgs<T> a;
  a.base = base;
  a.rs = rs;
  a.cs = cs;
  a.n = n;
  a.k = (int)k;
  a.kpad = kpad;
  a.J = J;
  a.Lf = Lf;
  a.ldl = ldl;
  a.Uf = Uf;
  a.ldu = ldu;
  a.diag = diag;
  a.slot_val = ws_ptr<uint64_t>(ctx, o_val);
  a.slot_idx = ws_ptr<int64_t>(ctx, o_idx);
  a.slot_row = ws_ptr<T>(ctx, o_row);
  a.flags = ws_ptr<unsigned>(ctx, o_flags);
  a.status = status_dev;

  RPID_CHECK(launch_fill_u64(ctx, a.slot_val, (size_t)k * G, kSentinel));
  RPID_CHECK(launch_fill_u64(ctx, reinterpret_cast<uint64_t*>(a.flags), 1, 0ull));
  if (ntmax == 256) return dispatch_R<T, 256>(ctx, a, R, G, nt);
  if (ntmax == 512) return dispatch_R<T, 512>(ctx, a, R, G, nt);
  return dispatch_R<T, 1024>(ctx, a, R, G, nt);
}

template int lupp_panel<double>(rpid_ctx, const double*, int64_t, int64_t, int64_t, int64_t,
                                int64_t*, double*, int64_t, double*, int64_t, double*, size_t,
                                int64_t*);
template int lupp_panel<float>(rpid_ctx, const float*, int64_t, int64_t, int64_t, int64_t,
                               int64_t*, float*, int64_t, float*, int64_t, float*, size_t,
                               int64_t*);

}  // namespace rpid
