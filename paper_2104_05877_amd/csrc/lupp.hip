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
//    the candidate's signed value into a per-step word; one wave of every
//    workgroup polls the G words of the step and reduces them identically
//    (largest |value|, ties to the smallest workgroup, which owns the
//    smallest rows), so every workgroup knows the winner and the pivot value
//    without a further exchange; thread j then reads word j of the winning
//    row (distinct addresses) while the multipliers are formed, and the
//    winning workgroup writes J, the pivot and row t of U from its own
//    registers.
//  * every exchanged word lives in uncached device memory, is written and
//    read with agent-scope atomics, and carries a tag (launch epoch, step) in
//    its upper 32 bits: a reader accepts a word only when its tag matches, so
//    nothing has to be ordered or flushed (an FP64 value travels as two
//    tagged halves).  Slots alternate between two buffers by step parity, so
//    a slot is rewritten only after every workgroup has read it.
//  One device-wide exchange per pivot; no second kernel launch per step.
#include <mutex>
#include <utility>
#include <vector>

#include "rpid_internal.hpp"

namespace rpid {

static constexpr unsigned kSpinLimit = 1u << 21;  // ~2 s of polling at ~1 us per load
// Every workgroup writes its candidate value into kValRep copies (64 KB
// apart) and reads copy g % kValRep, so the polls of the whole grid are
// spread over several memory channels instead of one region.
static constexpr int kValRep = 8;

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
  uint64_t* xval;   // [kValRep][2][G][W] tagged candidate values (replica stride xrep words)
  int64_t xrep;
  uint64_t* xrow;   // [2][G][kpad][W] tagged candidate rows
  uint64_t* xflag;  // [0] abort (tag = epoch)
  unsigned epoch;   // 1 .. 2^21 - 1
  int64_t* status;  // 0, t+1 (zero pivot), or a negative RPID_ERR code
};

template <typename T>
struct Words {
  static constexpr int W = sizeof(T) / 4;  // tagged words per value
};

__device__ __forceinline__ void wstore(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t wload(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned step_tag(unsigned epoch, int t) {
  return (epoch << 11) | (unsigned)(t + 1);
}

__device__ __forceinline__ void put_value(uint64_t* p, float v, unsigned tag) {
  wstore(p, ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v));
}
__device__ __forceinline__ void put_value(uint64_t* p, double v, unsigned tag) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  wstore(p, ((uint64_t)tag << 32) | (b >> 32));
  wstore(p + 1, ((uint64_t)tag << 32) | (b & 0xffffffffull));
}
__device__ __forceinline__ bool try_value(const uint64_t* p, unsigned tag, float& v) {
  const uint64_t w = wload(p);
  if ((unsigned)(w >> 32) != tag) return false;
  v = __uint_as_float((unsigned)w);
  return true;
}
__device__ __forceinline__ bool try_value(const uint64_t* p, unsigned tag, double& v) {
  const uint64_t w0 = wload(p), w1 = wload(p + 1);
  if ((unsigned)(w0 >> 32) != tag || (unsigned)(w1 >> 32) != tag) return false;
  v = __longlong_as_double((long long)((w0 << 32) | (w1 & 0xffffffffull)));
  return true;
}

// Value of a word set already known to carry the step's tag.
template <typename T>
__device__ __forceinline__ T word_value(const uint64_t* w);
template <>
__device__ __forceinline__ float word_value<float>(const uint64_t* w) {
  return __uint_as_float((unsigned)w[0]);
}
template <>
__device__ __forceinline__ double word_value<double>(const uint64_t* w) {
  return __longlong_as_double((long long)((w[0] << 32) | (w[1] & 0xffffffffull)));
}

// Spin until the tagged word(s) at p carry `tag`; false if the launch was
// aborted (another workgroup timed out) or this wait exceeded the spin limit.
template <typename V>
__device__ __forceinline__ bool wait_value(const uint64_t* p, unsigned tag, V& v, uint64_t* xflag,
                                           unsigned epoch) {
  unsigned spins = 0;
  while (!try_value(p, tag, v)) {
    if ((++spins & 255u) == 0) {
      if ((unsigned)wload(xflag) == epoch || spins > kSpinLimit) {
        wstore(xflag, (uint64_t)epoch);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
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

// R rows per thread, H threads per column (H = 2 for tall panels): workgroup
// g owns the R*H rows [g R H, (g+1) R H); thread tid = h * kpad + j holds
// column j of rows g R H + h R + q, q < R.
template <typename T, int R, int NTMAX, int H>
__global__ __launch_bounds__(NTMAX) void lupp_panel_kernel(LuppArgs<T> a) {
  constexpr int W = Words<T>::W;
  constexpr int RW = R * H;  // rows per workgroup
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int k = a.k;
  const int j = (H == 1) ? tid : tid % a.kpad;  // column of this thread
  const int h = (H == 1) ? 0 : tid / a.kpad;    // row part of this thread
  const int64_t row0 = (int64_t)g * RW;
  const int lane = tid & 63;
  const int wid = tid >> 6;

  __shared__ T colbuf[RW];  // column of the current step, this workgroup's rows
  __shared__ T mult[RW];    // multipliers of the current step (0 for frozen rows)
  __shared__ int alive[RW]; // 1 while the row has not been chosen as a pivot
  __shared__ T urow[H == 1 ? 1 : NTMAX / H];  // the candidate row (H > 1 only)
  __shared__ T cand_abs[H], cand_val[H];      // next step's candidate of each row part
  __shared__ int cand_row[H];
  __shared__ int sh_gw;
  __shared__ T sh_pv;
  __shared__ int sh_code;   // 0 go on, 1 stop: status in sh_status
  __shared__ int64_t sh_status;
  __shared__ int sh_abort;
  __shared__ int sh_bad;

  // ---- load this workgroup's rows of the panel into registers ------------
  // A row that has been a pivot is never read again (its U row is published
  // at its step and its later multipliers are 0), so its registers are set to
  // zero: the candidate search then needs no list of remaining rows (a zero
  // can only win where every remaining candidate is zero, which stops the
  // factorisation as an exactly zero pivot).  Rows beyond n load as zeros.
  T s[R];
  bool bad = false;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t row = row0 + h * R + q;
    T v = T(0);
    if (row < a.n && j < k) v = a.base[row * a.rs + (int64_t)j * a.cs];
    bad |= !isfinite(v);
    s[q] = v;
  }
  // the candidate of the owned column among this thread's rows (largest
  // modulus, the smallest row on ties), by a pairwise tree: a pair keeps its
  // right (larger-row) entry only if that entry is strictly larger
  auto local_candidate = [&]() {
    // runs of LC consecutive rows are scanned in order (a later row replaces
    // the run's best only if strictly larger), then the run winners go
    // through the pairwise tree: the same first-largest row as a tree over
    // all R rows, with 3 R / LC instead of 3 R values live at once
    constexpr int LC = R >= 64 ? 8 : 1;
    constexpr int NCH = R / LC;
    T av[NCH], sv[NCH];
    int iv[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      av[c] = fabs(s[c * LC]);
      sv[c] = s[c * LC];
      iv[c] = c * LC;
#pragma unroll
      for (int u = 1; u < LC; ++u) {
        const T x = fabs(s[c * LC + u]);
        const bool right = x > av[c];
        av[c] = right ? x : av[c];
        sv[c] = right ? s[c * LC + u] : sv[c];
        iv[c] = right ? c * LC + u : iv[c];
      }
    }
#pragma unroll
    for (int w = 1; w < NCH; w *= 2) {
#pragma unroll
      for (int q = 0; q + w < NCH; q += 2 * w) {
        const bool right = av[q + w] > av[q];
        av[q] = right ? av[q + w] : av[q];
        sv[q] = right ? sv[q + w] : sv[q];
        iv[q] = right ? iv[q + w] : iv[q];
      }
    }
    cand_abs[h] = av[0];
    cand_row[h] = h * R + iv[0];
    cand_val[h] = sv[0];
    return sv[0];
  };
  for (int q = tid; q < RW; q += nt) alive[q] = (row0 + q < a.n) ? 1 : 0;
  if (j == 0) {
#pragma unroll
    for (int q = 0; q < R; ++q) colbuf[h * R + q] = s[q];
    local_candidate();
  }
  if (tid == 0) {
    sh_abort = 0;
    sh_bad = 0;
  }
  __syncthreads();
  // a non-finite entry anywhere in the slab is published as a NaN candidate
  if (__any(bad && j < k) && lane == 0) sh_bad = 1;
  __syncthreads();

  int64_t final_status = 0;
  for (int t = 0; t < k; ++t) {
    const int par = t & 1;
    const unsigned tag = step_tag(a.epoch, t);
    // ---- (1) this workgroup's candidate (prepared at the end of last step) --
    int bq = cand_row[0];
    T best = cand_val[0];
    if (H > 1) {
      T ba = cand_abs[0];
#pragma unroll
      for (int p = 1; p < H; ++p) {
        if (cand_abs[p] > ba) {  // ties keep the earlier part (smaller rows)
          ba = cand_abs[p];
          bq = cand_row[p];
          best = cand_val[p];
        }
      }
    }
    if (t == 0 && sh_bad) best = T(NAN);

    // ---- (2) publish: candidate value, then the candidate row (tagged
    //      words; the value goes first so that it does not queue behind the
    //      row's stores).  With one thread per column the value of steps
    //      t > 0 went out already, from the owner of column t at the end of
    //      step t-1. ------------------------------------------------------------
    if (tid < kValRep && (H > 1 || t == 0))
      put_value(&a.xval[tid * a.xrep + ((int64_t)par * G + g) * W], best, tag);
    uint64_t* myrow = a.xrow + ((size_t)par * G + g) * a.kpad * W;
    T myv = T(0);  // this thread's column of the candidate row
    const int hb = bq / R, qb = bq - hb * R;
    if (h == hb && j >= t && j < k) {
#pragma unroll
      for (int q = 0; q < R; ++q) myv = (q == qb) ? s[q] : myv;
      if (j > t) put_value(myrow + (size_t)j * W, myv, tag);
      if (H > 1) urow[j] = myv;
    }

    // ---- (3) wave 0 gathers every workgroup's value and reduces ------------
    //      (all of a lane's words are requested at once, and a second round
    //      of requests is in flight while the first is checked)
    if (wid == 0) {
      T cv = T(-2), cpv = T(0);
      int ci = 0x7fffffff;
      bool ok = true, nonfinite = false;
      auto consider = [&](int i, T v) {
        if (!isfinite(v)) nonfinite = true;
        const T av = fabs(v);
        if (av > cv || (av == cv && i < ci)) {
          cv = av;
          ci = i;
          cpv = v;
        }
      };
      constexpr int PMAX = 4;
      if (G <= 64 * PMAX) {
        unsigned want = 0, got = 0, spins = 0;
#pragma unroll
        for (int c = 0; c < PMAX; ++c)
          if (lane + 64 * c < G) want |= 1u << c;
        T vals[PMAX];
        uint64_t wa[W * PMAX], wb[W * PMAX];
        // every round requests all PMAX words of the lane (indices past G
        // read word G-1 and are ignored): a fixed number of loads per round,
        // so the second round can stay in flight while the first is checked
        // the lane's words, addressed afresh per round (no pointer array kept
        // live beside the panel registers)
        const uint64_t* xw0 = &a.xval[(g % kValRep) * a.xrep + (int64_t)par * G * W];
        auto request = [&](uint64_t(&w)[W * PMAX]) {
#pragma unroll
          for (int c = 0; c < PMAX; ++c)
#pragma unroll
            for (int e = 0; e < W; ++e) w[c * W + e] = wload(xw0 + min(lane + 64 * c, G - 1) * W + e);
        };
        // accept the words of a set that carry this step's tag
        auto accept = [&](const uint64_t(&w)[W * PMAX], unsigned asked) {
#pragma unroll
          for (int c = 0; c < PMAX; ++c)
            if ((asked >> c) & 1u) {
              bool fresh = true;
#pragma unroll
              for (int e = 0; e < W; ++e) fresh &= (unsigned)(w[c * W + e] >> 32) == tag;
              if (fresh) {
                vals[c] = word_value<T>(&w[c * W]);
                got |= 1u << c;
              }
            }
        };
        request(wa);
        while (true) {
          request(wb);
          accept(wa, want & ~got);
          if (got == want) break;
          request(wa);
          accept(wb, want & ~got);
          if (got == want) break;
          if ((++spins & 127u) == 0) {
            if ((unsigned)wload(a.xflag) == a.epoch || spins > kSpinLimit / 2) {
              wstore(a.xflag, (uint64_t)a.epoch);
              ok = false;
              break;
            }
          }
        }
        // the set still in flight is not used again; wait for it before its
        // registers are reused
        __builtin_amdgcn_s_waitcnt(0);
        if (ok) {
#pragma unroll
          for (int c = 0; c < PMAX; ++c)
            if ((want >> c) & 1u) consider(lane + 64 * c, vals[c]);
        }
      } else {
        for (int i = lane; i < G && ok; i += 64) {
          T v;
          ok = wait_value(&a.xval[(g % kValRep) * a.xrep + ((int64_t)par * G + i) * W], tag, v,
                          a.xflag, a.epoch);
          if (ok) consider(i, v);
        }
      }
      const bool any_fail = __any(!ok);
      const bool any_nf = __any(nonfinite);
      // argmax over the wave carrying the signed value along
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const T ov = __shfl_xor(cv, off, 64);
        const int oi = __shfl_xor(ci, off, 64);
        const T opv = __shfl_xor(cpv, off, 64);
        const bool take = (ov > cv) || (ov == cv && oi < ci);
        cv = take ? ov : cv;
        ci = take ? oi : ci;
        cpv = take ? opv : cpv;
      }
      if (lane == 0) {
        sh_gw = ci;
        sh_pv = cpv;
        sh_code = 0;
        if (any_fail) {
          sh_code = 1;
          sh_status = RPID_ERR_TIMEOUT;
        } else if (any_nf) {
          sh_code = 1;
          sh_status = RPID_ERR_NONFINITE;
        } else if (!(cv > T(0))) {  // exactly zero pivot (or no candidate left)
          sh_code = 1;
          sh_status = t + 1;
        }
      }
    }
    __syncthreads();
    if (sh_code) {
      final_status = sh_status;
      break;
    }
    const int gw = sh_gw;
    const T pv = sh_pv;
    const bool winner = (g == gw);

    // ---- (4) multipliers, outputs, and the pivot row's words ---------------
    // the row words are requested first; the divisions overlap their latency
    T uj = T(0);
    bool ok = true;
    if (!winner && j > t && j < k)
      ok = wait_value(a.xrow + (((size_t)par * G + gw) * a.kpad + j) * W, tag, uj, a.xflag,
                      a.epoch);
    if (winner) uj = (H == 1) ? myv : urow[j < k ? j : 0];
    for (int q = tid; q < RW; q += nt) {
      const int64_t row = row0 + q;
      const bool is_piv = winner && q == bq;
      const bool live = alive[q] && !is_piv;
      const T mq = live ? colbuf[q] / pv : T(0);
      mult[q] = mq;
      if (row < a.n) a.Lf[row + (int64_t)t * a.ldl] = live ? mq : (is_piv ? T(1) : T(0));
    }
    if (winner) {
      if (tid == 0) {
        a.J[t] = row0 + bq;
        if (a.diag) a.diag[t] = fabs(pv);
      }
      if (h == 0 && j < k) a.Uf[t + (int64_t)j * a.ldu] = (j > t) ? uj : (j == t ? pv : T(0));
      if (h == hb) {
#pragma unroll
        for (int q = 0; q < R; ++q) s[q] = (q == qb) ? T(0) : s[q];
      }
    }
    if (!ok) sh_abort = 1;
    __syncthreads();
    if (sh_abort) {
      final_status = RPID_ERR_TIMEOUT;
      break;
    }

    // ---- (5) Schur update of this workgroup's rows, columns t+1..k-1; the
    //      owners of column t+1 mirror it and pick the next candidate --------
    if (winner && tid == 0) alive[bq] = 0;
    if (j > t && j < k) {
#pragma unroll
      for (int q = 0; q < R; ++q) s[q] = fma(-mult[h * R + q], uj, s[q]);
      if (j == t + 1) {
#pragma unroll
        for (int q = 0; q < R; ++q) colbuf[h * R + q] = s[q];
        const T nv = local_candidate();
        if (H == 1 && t + 1 < k) {
          // the workgroup's candidate of step t+1 is this thread's: publish
          // it now rather than after the barrier (its slot was last read in
          // step t-1, which every workgroup has finished polling by the time
          // any workgroup has seen all values of step t)
          const int64_t at = ((int64_t)((t + 1) & 1) * G + g) * W;
          const unsigned tag1 = step_tag(a.epoch, t + 1);
#pragma unroll
          for (int r = 0; r < kValRep; ++r) put_value(&a.xval[r * a.xrep + at], nv, tag1);
        }
      }
    }
    __syncthreads();
  }
  if (g == 0 && tid == 0) *a.status = final_status;
}

size_t lupp_workspace_bytes(rpid_ctx ctx, int64_t n, int64_t k, int elem_bytes) {
  // the exchange slots live in the context's uncached buffer
  (void)ctx;
  (void)n;
  (void)k;
  (void)elem_bytes;
  return 256;
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
static constexpr int row_reg_budget(int ntmax) { return ntmax <= 768 ? 160 : 80; }

template <typename T, int R, int NTMAX, int H>
static int launch_lupp_R(rpid_ctx ctx, LuppArgs<T> a, int G, int nt) {
  if constexpr (R * (int)sizeof(T) / 4 > row_reg_budget(NTMAX)) {
    return RPID_ERR_UNSUPPORTED;
  } else {
    void* kargs[] = {&a};
    const void* fn = reinterpret_cast<const void*>(lupp_panel_kernel<T, R, NTMAX, H>);
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

template <typename T, int NTMAX, int H>
static int dispatch_R(rpid_ctx ctx, LuppArgs<T> a, int R, int G, int nt) {
  switch (R) {
    case 16: return launch_lupp_R<T, 16, NTMAX, H>(ctx, a, G, nt);
    case 32: return launch_lupp_R<T, 32, NTMAX, H>(ctx, a, G, nt);
    case 64: return launch_lupp_R<T, 64, NTMAX, H>(ctx, a, G, nt);
    case 128: return launch_lupp_R<T, 128, NTMAX, H>(ctx, a, G, nt);
    default: return RPID_ERR_UNSUPPORTED;
  }
}

// Uncached exchange buffers are never freed once a kernel has read them, so
// they are pooled per device for the life of the process: a context takes one
// at its first pivoting call and hands it back in rpid_destroy, so contexts
// created in a loop reuse the same few buffers.  Each buffer carries its
// launch epoch with it (the tag of the words its latest launch wrote), so a
// launch on a recycled buffer never takes a stale word for a fresh one.
namespace {
struct UcBuffer {
  void* p = nullptr;
  size_t bytes = 0;
  unsigned epoch = 0;
};
std::mutex g_uc_mu;
std::vector<std::pair<int, UcBuffer>> g_uc_pool;  // (device, buffer), free buffers
}  // namespace

void release_exchange_buffer(rpid_ctx ctx) {
  if (!ctx->uc) return;
  std::lock_guard<std::mutex> lk(g_uc_mu);
  g_uc_pool.push_back({ctx->device, UcBuffer{ctx->uc, ctx->uc_bytes, ctx->lupp_epoch}});
  ctx->uc = nullptr;
  ctx->uc_bytes = 0;
  ctx->lupp_epoch = 0;
}

// The context's uncached exchange buffer, at least `bytes` long, and a fresh
// launch epoch for the tags; a buffer is cleared when it is new or its epoch
// wraps.  A buffer that is too small goes back to the pool (still allocated).
static int exchange_buffer(rpid_ctx ctx, size_t bytes, char** base, unsigned* epoch) {
  bool fresh = false;
  if (bytes > ctx->uc_bytes) {
    release_exchange_buffer(ctx);
    {
      std::lock_guard<std::mutex> lk(g_uc_mu);
      for (size_t i = 0; i < g_uc_pool.size(); ++i) {
        if (g_uc_pool[i].first == ctx->device && g_uc_pool[i].second.bytes >= bytes) {
          ctx->uc = g_uc_pool[i].second.p;
          ctx->uc_bytes = g_uc_pool[i].second.bytes;
          ctx->lupp_epoch = g_uc_pool[i].second.epoch;
          g_uc_pool.erase(g_uc_pool.begin() + i);
          break;
        }
      }
    }
    if (!ctx->uc) {
      size_t want = bytes < ((size_t)4 << 20) ? ((size_t)4 << 20) : bytes;
      void* p = nullptr;
      if (hipExtMallocWithFlags(&p, want, hipDeviceMallocUncached) != hipSuccess) return RPID_ERR_NOMEM;
      ctx->uc = p;
      ctx->uc_bytes = want;
      ctx->lupp_epoch = 0;
      fresh = true;
    }
  }
  // launch epoch (21 bits) tags every exchanged word; tag 0 never matches
  if (++ctx->lupp_epoch >= (1u << 21)) {
    ctx->lupp_epoch = 1;
    fresh = true;
  }
  if (fresh) RPID_CHECK(launch_fill_u64(ctx, static_cast<uint64_t*>(ctx->uc), ctx->uc_bytes / 8, 0ull));
  *base = static_cast<char*>(ctx->uc);
  *epoch = ctx->lupp_epoch;
  return RPID_OK;
}

template <typename T>
int lupp_panel(rpid_ctx ctx, const T* base, int64_t rs, int64_t cs, int64_t n, int64_t k,
               int64_t* J, T* Lf, int64_t ldl, T* Uf, int64_t ldu, T* diag, size_t ws_off,
               int64_t* status_dev) {
  if (k < 1 || k > 1024 || n < k) return RPID_ERR_UNSUPPORTED;
  const int kpad = (int)((k + 63) / 64 * 64);
  // Rows per thread: the smallest R whose grid fits one workgroup per CU (more
  // rows cost registers, fewer cost polling), capped by the register budget.
  auto pick = [&](int ntmax, int h, int& R, int64_t& G) {
    const int rmax = max_rows(ntmax, (int)sizeof(T));
    R = rmax;
    for (int c = 16; c <= rmax; c *= 2) {
      if ((n + (int64_t)c * h - 1) / ((int64_t)c * h) <= ctx->num_cu) {
        R = c;
        break;
      }
    }
    G = (n + (int64_t)R * h - 1) / ((int64_t)R * h);
  };
  int H = 1, nt = kpad;
  int ntmax = nt <= 256 ? 256 : (nt <= 512 ? 512 : 1024);
  int R;
  int64_t G64;
  pick(ntmax, 1, R, G64);
  if (G64 > ctx->num_cu && 2 * kpad <= 1024) {
    // tall panel: two threads per column keep one workgroup per CU
    const int nt2 = 2 * kpad;
    const int ntmax2 = nt2 <= 512 ? 512 : (nt2 <= 768 ? 768 : 1024);
    int R2;
    int64_t G2;
    pick(ntmax2, 2, R2, G2);
    if (G2 < G64) {
      H = 2;
      nt = nt2;
      ntmax = ntmax2;
      R = R2;
      G64 = G2;
    }
  }
  // One workgroup per compute unit at most.  A grid of two workgroups per CU
  // once ran into the spin limit of the exchange (the 384 x 65536 FP32 panel,
  // before it moved to two threads per column) and the cause is not known, so
  // such grids are refused rather than launched.
  if (G64 > ctx->num_cu) return RPID_ERR_UNSUPPORTED;
  const int G = (int)G64;
  const int xstride = kpad;  // words per published row

  (void)ws_off;
  constexpr int W = Words<T>::W;
  Carve cv;
  // value copies 64 KB apart (or further, for large grids)
  const int64_t xrep = ((int64_t)2 * G * W + 8191) / 8192 * 8192;
  const size_t o_val = cv.take<uint64_t>((size_t)kValRep * xrep);
  const size_t o_row = cv.take<uint64_t>((size_t)2 * G * xstride * W);
  const size_t o_flag = cv.take<uint64_t>(1);
  char* ucb = nullptr;
  unsigned epoch = 0;
  RPID_CHECK(exchange_buffer(ctx, cv.off, &ucb, &epoch));

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
  a.xval = reinterpret_cast<uint64_t*>(ucb + o_val);
  a.xrep = xrep;
  a.xrow = reinterpret_cast<uint64_t*>(ucb + o_row);
  a.xflag = reinterpret_cast<uint64_t*>(ucb + o_flag);
  a.epoch = epoch;
  a.status = status_dev;
  if (H == 1) {
    if (ntmax == 256) return dispatch_R<T, 256, 1>(ctx, a, R, G, nt);
    if (ntmax == 512) return dispatch_R<T, 512, 1>(ctx, a, R, G, nt);
    return dispatch_R<T, 1024, 1>(ctx, a, R, G, nt);
  }
  if (ntmax == 512) return dispatch_R<T, 512, 2>(ctx, a, R, G, nt);
  if (ntmax == 768) return dispatch_R<T, 768, 2>(ctx, a, R, G, nt);
  return dispatch_R<T, 1024, 2>(ctx, a, R, G, nt);
}

template int lupp_panel<double>(rpid_ctx, const double*, int64_t, int64_t, int64_t, int64_t,
                                int64_t*, double*, int64_t, double*, int64_t, double*, size_t,
                                int64_t*);
template int lupp_panel<float>(rpid_ctx, const float*, int64_t, int64_t, int64_t, int64_t,
                               int64_t*, float*, int64_t, float*, int64_t, float*, size_t,
                               int64_t*);

// ---------------------------------------------------------------------------
// Column-pivoted Householder QR of a sketch X (l x n), k steps, as one
// persistent cooperative kernel (the CPQR of eq. def_QRCP, applied to the
// sketch as in Rand-CPQR).
//
// Panel P(i, j) = base[i * rs + j * cs] = X(j, i): i = column of X (the
// candidate), j = row of X.  Workgroup g owns candidates [g R, g R + R);
// thread j (< l) holds P(i, j) of them in R registers.
// Step t: pivot p_t = the remaining column with the largest norm of its
// rows t..l-1 (ties to the smallest column); Householder reflector from the
// pivot column, w = X(t:l, p_t): alpha = -sign(w_0) ||w||, v = w - alpha e_0,
// H = I - beta v v^T with beta = 1 / (alpha (alpha - w_0)); every remaining
// column gets x <- x - beta (v^T x) v.  Row t of R is the updated row t
// (R(t, p_t) = alpha); the column norms of rows t+1.. are recomputed from the
// updated values (no downdating).
// Exchange per step as in the LUPP kernel: a tagged candidate value (the
// squared norm) in kValRep copies, the candidate column as tagged words,
// one wave per workgroup polls and reduces the values identically.  Every
// workgroup builds alpha and beta from the same fetched words in the same
// order, so all of them apply bit-identical reflectors.
// Sums over the l rows of a column (the dot products v^T x and the norms)
// are workgroup reductions of R values at once: within a wave, halving
// exchanges leave lane pair (2q, 2q+1) (R = 32) with the wave's sum for
// candidate q, then the per-wave sums are added in wave order.
template <typename T>
struct CpqrArgs {
  const T* base;
  int64_t rs, cs;
  int64_t n;
  int l, lpad, k;
  int64_t* J;
  T* Rf;
  int64_t ldr;
  T* diag;
  uint64_t* xval;
  int64_t xrep;
  uint64_t* xrow;
  uint64_t* xflag;
  unsigned epoch;
  int64_t* status;
};

// One halving exchange of wave_rowsum: C values per lane become C / 2, the
// lane keeping the upper half when its bit O is set (O = 32 C / R), and the
// next exchange follows.  Recursion keeps every register index a constant.
template <typename T, int C, int R>
struct RowsumHalve {
  static __device__ __forceinline__ void run(T* v, int lane) {
    constexpr int H = C / 2;
    constexpr int O = 32 * C / R;
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const T send = up ? v[i] : v[H + i];
      const T keep = up ? v[H + i] : v[i];
      v[i] = keep + __shfl_xor(send, O, 64);
    }
    RowsumHalve<T, H, R>::run(v, lane);
  }
};
template <typename T, int R>
struct RowsumHalve<T, 1, R> {
  static __device__ __forceinline__ void run(T*, int) {}
};

// Sum over the 64 lanes of a wave for each of R values per lane; the result
// for value q ends in lanes q * (64 / R) .. (q + 1) * (64 / R) - 1.
template <typename T, int R>
__device__ __forceinline__ T wave_rowsum(T (&v)[R], int lane) {
  static_assert(R >= 1 && R <= 64 && (R & (R - 1)) == 0, "R a power of two <= 64");
  RowsumHalve<T, R, R>::run(v, lane);
#pragma unroll
  for (int o = 32 / R; o >= 1; o /= 2) v[0] += __shfl_xor(v[0], o, 64);
  return v[0];
}

template <typename T, int R, int NTMAX>
__global__ __launch_bounds__(NTMAX) void cpqr_panel_kernel(CpqrArgs<T> a) {
  constexpr int W = Words<T>::W;
  constexpr int NW = NTMAX / 64;
  const int tid = threadIdx.x;
  const int nwav = blockDim.x / 64;
  const int g = blockIdx.x;
  const int G = gridDim.x;
  const int l = a.l, k = a.k;
  const int j = tid;  // row of X held by this thread
  const int64_t row0 = (int64_t)g * R;
  const int lane = tid & 63;
  const int wid = tid >> 6;

  __shared__ T part[NW][R];
  __shared__ T nrm[R];
  __shared__ T dsum[R];
  __shared__ int alive[R];
  __shared__ T wpart[NW];
  __shared__ T sh_w0;
  __shared__ int sh_bq, sh_gw, sh_code, sh_abort, sh_bad;
  __shared__ T sh_best;
  __shared__ int64_t sh_status;

  T s[R];
  bool bad = false;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t col = row0 + q;
    T v = T(0);
    if (col < a.n && j < l) v = a.base[col * a.rs + (int64_t)j * a.cs];
    bad |= !isfinite(v);
    s[q] = v;
  }
  for (int q = tid; q < R; q += blockDim.x) alive[q] = (row0 + q < a.n) ? 1 : 0;
  if (tid == 0) {
    sh_abort = 0;
    sh_bad = 0;
  }
  __syncthreads();
  if (__any(bad) && lane == 0) sh_bad = 1;

  // out[q] = sum over the threads of vals[q] (wave sums added in wave order)
  auto block_rowsum = [&](T (&vals)[R], T* out) {
    const T ws = wave_rowsum<T, R>(vals, lane);
    if ((lane & (64 / R - 1)) == 0) part[wid][lane / (64 / R)] = ws;
    __syncthreads();
    if (tid < R) {
      T acc = part[0][tid];
      for (int w = 1; w < nwav; ++w) acc += part[w][tid];
      out[tid] = acc;
    }
    __syncthreads();
  };
  // squared norms of rows t.. of every owned column, and the candidate
  auto norms_and_candidate = [&](int t) {
    T vals[R];
#pragma unroll
    for (int q = 0; q < R; ++q) vals[q] = (j >= t && j < l) ? s[q] * s[q] : T(0);
    block_rowsum(vals, nrm);
    if (wid == 0) {
      T v = (lane < R && alive[lane]) ? nrm[lane] : T(-1);
      int i = lane < R ? lane : 0x7fffffff;
      wave_argmax(v, i);
      if (lane == 0) {
        sh_bq = i;
        sh_best = v;
      }
    }
    __syncthreads();
  };
  norms_and_candidate(0);

  int64_t final_status = 0;
  for (int t = 0; t < k; ++t) {
    const int par = t & 1;
    const unsigned tag = step_tag(a.epoch, t);
    const int bq = sh_bq;
    T best = sh_best;  // -1 when no column is left here
    if (t == 0 && sh_bad) best = T(NAN);

    // ---- publish the candidate's squared norm, then its rows t.. --------
    if (tid < kValRep) put_value(&a.xval[tid * a.xrep + ((int64_t)par * G + g) * W], best, tag);
    uint64_t* mycol = a.xrow + ((size_t)par * G + g) * a.lpad * W;
    T myv = T(0);
#pragma unroll
    for (int q = 0; q < R; ++q) myv = (q == bq) ? s[q] : myv;
    if (j >= t && j < l) put_value(mycol + (size_t)j * W, myv, tag);

    // ---- wave 0 gathers every workgroup's value and reduces (each lane
    //      requests all of its words at once, G <= 256) --------------------
    if (wid == 0) {
      T cv = T(-2);
      int ci = 0x7fffffff;
      bool ok = true, nonfinite = false;
      constexpr int PMAX = 4;
      unsigned want = 0, got = 0, spins = 0;
#pragma unroll
      for (int c = 0; c < PMAX; ++c)
        if (lane + 64 * c < G) want |= 1u << c;
      const uint64_t* xw[PMAX];
#pragma unroll
      for (int c = 0; c < PMAX; ++c)
        xw[c] = &a.xval[(g % kValRep) * a.xrep + ((int64_t)par * G + min(lane + 64 * c, G - 1)) * W];
      T vals[PMAX];
      while (got != want) {
        uint64_t wv[W * PMAX];
#pragma unroll
        for (int c = 0; c < PMAX; ++c)
#pragma unroll
          for (int e = 0; e < W; ++e) wv[c * W + e] = wload(xw[c] + e);
#pragma unroll
        for (int c = 0; c < PMAX; ++c)
          if (((want & ~got) >> c) & 1u) {
            bool fresh = true;
#pragma unroll
            for (int e = 0; e < W; ++e) fresh &= (unsigned)(wv[c * W + e] >> 32) == tag;
            if (fresh) {
              vals[c] = word_value<T>(&wv[c * W]);
              got |= 1u << c;
            }
          }
        if (got != want && (++spins & 127u) == 0) {
          if ((unsigned)wload(a.xflag) == a.epoch || spins > kSpinLimit / 2) {
            wstore(a.xflag, (uint64_t)a.epoch);
            ok = false;
            break;
          }
        }
      }
      if (ok) {
#pragma unroll
        for (int c = 0; c < PMAX; ++c)
          if ((want >> c) & 1u) {
            const T v = vals[c];
            const int i = lane + 64 * c;
            if (!isfinite(v)) nonfinite = true;
            if (v > cv || (v == cv && i < ci)) {
              cv = v;
              ci = i;
            }
          }
      }
      const bool any_fail = __any(!ok);
      const bool any_nf = __any(nonfinite);
      wave_argmax(cv, ci);
      if (lane == 0) {
        sh_gw = ci;
        sh_code = 0;
        if (any_fail) {
          sh_code = 1;
          sh_status = RPID_ERR_TIMEOUT;
        } else if (any_nf) {
          sh_code = 1;
          sh_status = RPID_ERR_NONFINITE;
        } else if (!(cv > T(0))) {  // every remaining column is zero in rows t..
          sh_code = 1;
          sh_status = t + 1;
        }
      }
    }
    __syncthreads();
    if (sh_code) {
      final_status = sh_status;
      break;
    }
    const int gw = sh_gw;
    const bool winner = (g == gw);

    // ---- the pivot column's rows t.., its norm, the reflector ------------
    T w = T(0);
    bool ok = true;
    if (j >= t && j < l) {
      if (winner)
        w = myv;
      else
        ok = wait_value(a.xrow + (((size_t)par * G + gw) * a.lpad + j) * W, tag, w, a.xflag, a.epoch);
    }
    if (!ok) sh_abort = 1;
    {
      T w2 = w * w;
#pragma unroll
      for (int o = 32; o >= 1; o /= 2) w2 += __shfl_xor(w2, o, 64);
      if (lane == 0) wpart[wid] = w2;
      if (j == t) sh_w0 = w;
    }
    __syncthreads();
    if (sh_abort) {
      final_status = RPID_ERR_TIMEOUT;
      break;
    }
    // every thread forms alpha and beta from the same values in the same order
    T nw2 = wpart[0];
    for (int i = 1; i < nwav; ++i) nw2 += wpart[i];
    const T w0 = sh_w0;
    const T nw = sqrt(nw2);
    const T alpha = (w0 >= T(0)) ? -nw : nw;
    const T beta = T(1) / (alpha * (alpha - w0));
    const T vj = (j == t) ? w - alpha : ((j > t && j < l) ? w : T(0));

    // ---- v^T x for every owned column, then x <- x - beta (v^T x) v -------
    {
      T vals[R];
#pragma unroll
      for (int q = 0; q < R; ++q) vals[q] = vj * s[q];
      block_rowsum(vals, dsum);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) s[q] = fma(-beta * dsum[q], vj, s[q]);
    // row t of R: the updated row t (alpha at the pivot, 0 for earlier
    // pivots).  Thread t is the only reader of `alive` until the next
    // reduction's barrier, so it also retires the pivot.
    if (j == t) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int64_t col = row0 + q;
        if (col < a.n) {
          const bool is_piv = winner && q == bq;
          a.Rf[t + col * a.ldr] = is_piv ? alpha : (alive[q] ? s[q] : T(0));
        }
      }
      if (winner) alive[bq] = 0;
    }
    if (winner) {
      if (tid == 0) {
        a.J[t] = row0 + bq;
        if (a.diag) a.diag[t] = fabs(alpha);
      }
#pragma unroll
      for (int q = 0; q < R; ++q) s[q] = (q == bq) ? T(0) : s[q];
    }
    if (t + 1 < k) norms_and_candidate(t + 1);
  }
  if (g == 0 && tid == 0) *a.status = final_status;
}

template <typename T, int R, int NTMAX>
static int launch_cpqr(rpid_ctx ctx, CpqrArgs<T> a, int G, int nt) {
  void* kargs[] = {&a};
  const void* fn = reinterpret_cast<const void*>(cpqr_panel_kernel<T, R, NTMAX>);
  int per_cu = 0;
  RPID_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, 0));
  if (per_cu < 1 || (int64_t)per_cu * ctx->num_cu < G) return RPID_ERR_LAUNCH;
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(nt), kargs, 0, ctx->stream);
  if (e != hipSuccess) return RPID_ERR_LAUNCH;
  return RPID_OK;
}

// R = 16 or 32 columns per workgroup and at most 512 threads keep the
// column values, the reduction operands and the temporaries in registers.
template <typename T, int NTMAX>
static int cpqr_dispatch_R(rpid_ctx ctx, CpqrArgs<T> a, int R, int G, int nt) {
  switch (R) {
    case 16: return launch_cpqr<T, 16, NTMAX>(ctx, a, G, nt);
    case 32: return launch_cpqr<T, 32, NTMAX>(ctx, a, G, nt);
    default: return RPID_ERR_UNSUPPORTED;
  }
}

template <typename T>
int cpqr_panel(rpid_ctx ctx, const T* base, int64_t rs, int64_t cs, int64_t n, int64_t l, int64_t k,
               int64_t* J, T* Rf, int64_t ldr, T* diag, int64_t* status_dev) {
  if (l < 1 || l > 512 || k < 1 || k > l || k > n) return RPID_ERR_UNSUPPORTED;
  const int lpad = (int)((l + 63) / 64 * 64);
  const int ntmax = lpad <= 256 ? 256 : 512;
  int R = 32;
  for (int c = 16; c <= 32; c *= 2)
    if ((n + c - 1) / c <= ctx->num_cu) {
      R = c;
      break;
    }
  const int64_t G64 = (n + R - 1) / R;
  if (G64 > ctx->num_cu || G64 > 256) return RPID_ERR_UNSUPPORTED;  // the poll covers 4 x 64 values
  const int G = (int)G64;
  constexpr int W = Words<T>::W;
  Carve cv;
  const int64_t xrep = ((int64_t)2 * G * W + 8191) / 8192 * 8192;
  const size_t o_val = cv.take<uint64_t>((size_t)kValRep * xrep);
  const size_t o_row = cv.take<uint64_t>((size_t)2 * G * lpad * W);
  const size_t o_flag = cv.take<uint64_t>(1);
  char* ucb = nullptr;
  unsigned epoch = 0;
  RPID_CHECK(exchange_buffer(ctx, cv.off, &ucb, &epoch));
  CpqrArgs<T> a;
  a.base = base;
  a.rs = rs;
  a.cs = cs;
  a.n = n;
  a.l = (int)l;
  a.lpad = lpad;
  a.k = (int)k;
  a.J = J;
  a.Rf = Rf;
  a.ldr = ldr;
  a.diag = diag;
  a.xval = reinterpret_cast<uint64_t*>(ucb + o_val);
  a.xrep = xrep;
  a.xrow = reinterpret_cast<uint64_t*>(ucb + o_row);
  a.xflag = reinterpret_cast<uint64_t*>(ucb + o_flag);
  a.epoch = epoch;
  a.status = status_dev;
  if (ntmax == 256) return cpqr_dispatch_R<T, 256>(ctx, a, R, G, lpad);
  return cpqr_dispatch_R<T, 512>(ctx, a, R, G, lpad);
}

template int cpqr_panel<double>(rpid_ctx, const double*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                int64_t*, double*, int64_t, double*, int64_t*);
template int cpqr_panel<float>(rpid_ctx, const float*, int64_t, int64_t, int64_t, int64_t, int64_t,
                               int64_t*, float*, int64_t, float*, int64_t*);

}  // namespace rpid
