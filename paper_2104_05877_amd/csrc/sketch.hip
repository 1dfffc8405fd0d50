// Row sketch X = Omega A (Alg. 2, step 2) on the MFMA units of gfx950.
//
// Operands: Pt (= Omega^T) is m x l column-major, so every row of Omega is
// contiguous along m; A is m x n column-major.  X(r, j) = sum_i Pt(i, r) A(i, j).
//
// Tiling (one workgroup = 4 waves):
//  * a workgroup produces all rows of one l-chunk (up to 16*RT rows) for a
//    strip of 4*CT*16 columns, over one K-range (split-K);
//  * A is the streamed operand: each lane loads VEC consecutive elements of
//    one column (16 or 32 bytes) straight into the MFMA B-operand register;
//    the MFMA k-slots are permuted so that these VEC values are the lane's
//    k-values of VEC consecutive MFMAs (the reduction order does not change
//    the result beyond rounding);
//  * Omega chunks (16*RT rows x BK) are staged in LDS, double buffered, and
//    shared by the 4 waves;
//  * split-K partial sums go to a workspace and a second kernel adds them in
//    a fixed order (deterministic).
// The K-range index is the fastest-varying part of the workgroup id, so the
// workgroups that share an Omega slice land on the same XCD (round-robin
// dispatch) and keep that slice in the XCD's L2.
#include "rpid_internal.hpp"

namespace rpid {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

// Per-dtype traits: element storage, vector width per lane, accumulator.
template <typename TE>
struct MT;
template <>
struct MT<double> {
  using Acc = double;
  using AccV = v4d;
  static constexpr int VEC = 4;     // elements per lane load (4 MFMA k-steps of 1)
  static constexpr int KMFMA = 1;   // k-values per lane per MFMA
  static constexpr int BK = 16;     // K per LDS stage (LDS: 272 x 20 x 8 B x 2)
  static constexpr int CT = 2;      // column tiles per wave
  // accumulator register i of lane-group q holds row q + 4 i of the tile
  static __device__ __forceinline__ int out_row(int q, int i) { return q + 4 * i; }
};
template <>
struct MT<float> {
  using Acc = float;
  using AccV = v4f;
  static constexpr int VEC = 4;
  static constexpr int KMFMA = 1;
  static constexpr int BK = 32;
  static constexpr int CT = 3;
  // accumulator register i of lane-group q holds row 4 q + i of the tile
  static __device__ __forceinline__ int out_row(int q, int i) { return 4 * q + i; }
};
template <>
struct MT<uint16_t> {  // bf16 storage
  using Acc = float;
  using AccV = v4f;
  static constexpr int VEC = 8;
  static constexpr int KMFMA = 8;
  static constexpr int BK = 64;
  static constexpr int CT = 3;
  static __device__ __forceinline__ int out_row(int q, int i) { return 4 * q + i; }
};

template <>
struct MT<uint8_t> {  // OCP E4M3 storage (FP8)
  using Acc = float;
  using AccV = v4f;
  static constexpr int VEC = 32;    // 32 bytes per lane: the lane's k-values of one MFMA
  static constexpr int KMFMA = 32;
  static constexpr int BK = 128;
  static constexpr int CT = 2;      // 32-byte fragments leave room for two column tiles
  // same output layout as the BF16 MFMA: register i of lane-group q is row 4 q + i
  static __device__ __forceinline__ int out_row(int q, int i) { return 4 * q + i; }
};

template <typename TE>
struct Frag {
  TE v[MT<TE>::VEC];
};

template <typename TE>
__device__ __forceinline__ typename MT<TE>::AccV mfma_step(const Frag<TE>& a, const Frag<TE>& b,
                                                           int s, typename MT<TE>::AccV c);
template <>
__device__ __forceinline__ v4d mfma_step<double>(const Frag<double>& a, const Frag<double>& b,
                                                 int s, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[s], b.v[s], c, 0, 0, 0);
}
template <>
__device__ __forceinline__ v4f mfma_step<float>(const Frag<float>& a, const Frag<float>& b, int s,
                                                v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[s], b.v[s], c, 0, 0, 0);
}
template <>
__device__ __forceinline__ v4f mfma_step<uint16_t>(const Frag<uint16_t>& a,
                                                   const Frag<uint16_t>& b, int s, v4f c) {
  (void)s;
  v8bf av, bv;
  __builtin_memcpy(&av, a.v, 16);
  __builtin_memcpy(&bv, b.v, 16);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
}

template <>
__device__ __forceinline__ v4f mfma_step<uint8_t>(const Frag<uint8_t>& a, const Frag<uint8_t>& b,
                                                  int s, v4f c) {
  (void)s;
  v8i av, bv;
  __builtin_memcpy(&av, a.v, 32);
  __builtin_memcpy(&bv, b.v, 32);
  // both operands E4M3 (format selectors 0), no block scales
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 0, 0, 0, 0, 0, 0);
}

template <typename TE>
__device__ __forceinline__ void load_frag(Frag<TE>& f, const TE* p) {
  static_assert(sizeof(Frag<TE>) % 16 == 0, "fragment must be whole 16-byte vectors");
  const uint4* src = reinterpret_cast<const uint4*>(p);
  uint4* dst = reinterpret_cast<uint4*>(f.v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(Frag<TE>) / 16); ++i) dst[i] = src[i];
}

template <typename TE>
__device__ __forceinline__ void load_frag_guarded(Frag<TE>& f, const TE* col, int64_t k,
                                                  int64_t m) {
#pragma unroll
  for (int i = 0; i < MT<TE>::VEC; ++i) f.v[i] = (k + i < m) ? col[k + i] : TE(0);
}

template <typename TE>
struct SketchArgs {
  const TE* Pt;
  int64_t ldp;
  const TE* A;
  int64_t lda;
  int64_t m, n;
  int l;
  int split;       // number of K-ranges
  int64_t kchunk;  // K per range (multiple of BK)
  int ltiles;      // row tiles (of 16) per l-chunk
  typename MT<TE>::Acc* out;  // split-K partials (split slices of l x n) or X itself
  int64_t ldo;                // leading dimension of out (rows)
  int64_t out_split_stride;   // elements between split slices (0 if split == 1)
  int64_t kpairs;             // streaming kernel: K in stages, shared out evenly
  int vec_out;                // streaming kernel: out rows writable as 4-element vectors
  // residual epilogue: R (l x n, BF16) minus the product, squared and summed
  const uint16_t* R;
  int64_t ldr;
  int vec_r;                  // 4 consecutive rows of R are one 8-byte load
  double* partials;           // [grid][2]: sum (R - product)^2, sum R^2
};

template <typename TE, int RT, bool ALIGNED>
__global__ __launch_bounds__(256) void sketch_kernel(SketchArgs<TE> a) {
  using M = MT<TE>;
  using AccV = typename M::AccV;
  constexpr int VEC = M::VEC;
  constexpr int BK = M::BK;
  constexpr int CT = M::CT;
  constexpr int SUB = BK / (4 * VEC);        // lane-loads per column per stage
  constexpr int LROW = BK + 16 / (int)sizeof(TE) * 2;  // padded LDS row (elements)
  constexpr int ROWS = 16 * RT;

  __shared__ __attribute__((aligned(16))) TE lds[2][ROWS * LROW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int q = lane >> 4;   // k-slot group
  const int c16 = lane & 15;

  // workgroup -> (split, column strip, l-chunk); split fastest (XCD-aware)
  const int bid = blockIdx.x;
  const int split_id = bid % a.split;
  const int rest = bid / a.split;
  const int64_t ncolstrips = (a.n + 4 * CT * 16 - 1) / (4 * CT * 16);
  const int strip = (int)(rest % ncolstrips);
  const int lchunk = (int)(rest / ncolstrips);

  const int row_base = lchunk * ROWS;
  const int64_t kbeg = (int64_t)split_id * a.kchunk;
  const int64_t kend = min(a.m, kbeg + a.kchunk);
  const int64_t col_base = (int64_t)strip * (4 * CT * 16) + wid * (CT * 16);

  AccV acc[RT][CT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = AccV{};

  // Stage an Omega chunk [row_base, row_base + ROWS) x [k0, k0 + BK) into LDS.
  auto stage = [&](int buf, int64_t k0) {
    constexpr int EPV = 16 / (int)sizeof(TE);  // elements per 16-byte vector
    constexpr int VPR = BK / EPV;               // vectors per row
    for (int v = tid; v < ROWS * VPR; v += 256) {
      const int r = v / VPR;
      const int kk = (v % VPR) * EPV;
      const int grow = row_base + r;
      TE* dst = &lds[buf][r * LROW + kk];
      if (grow < a.l && ALIGNED && k0 + kk + EPV <= kend) {
        *reinterpret_cast<uint4*>(dst) =
            *reinterpret_cast<const uint4*>(a.Pt + (int64_t)grow * a.ldp + k0 + kk);
      } else {
#pragma unroll
        for (int e = 0; e < EPV; ++e) {
          const int64_t kg = k0 + kk + e;
          dst[e] = (grow < a.l && kg < kend) ? a.Pt[(int64_t)grow * a.ldp + kg] : TE(0);
        }
      }
    }
  };

  if (kbeg < kend) stage(0, kbeg);
  int buf = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    if (k0 + BK < kend) stage(buf ^ 1, k0 + BK);
    const bool full = ALIGNED && (k0 + BK <= kend);
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub) {
      // B-operand fragments (columns of A) for this sub-step
      Frag<TE> bf[CT];
      const int64_t kk = k0 + sub * 4 * VEC + q * VEC;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int64_t col = col_base + c * 16 + c16;
        if (col < a.n) {
          const TE* cp = a.A + col * a.lda;
          if (full)
            load_frag(bf[c], cp + kk);
          else
            load_frag_guarded(bf[c], cp, kk, kend);
        } else {
#pragma unroll
          for (int i = 0; i < VEC; ++i) bf[c].v[i] = TE(0);
        }
      }
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        Frag<TE> af;
        load_frag(af, &lds[buf][(r * 16 + c16) * LROW + sub * 4 * VEC + q * VEC]);
#pragma unroll
        for (int s = 0; s < VEC / M::KMFMA; ++s)
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[r][c] = mfma_step<TE>(af, bf[c], s, acc[r][c]);
      }
    }
    buf ^= 1;
  }

  // Write the tile: acc[r][c][i] is row 16r + out_row(q, i), column 16c + c16.
  typename M::Acc* out = a.out + (int64_t)split_id * a.out_split_stride;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int64_t col = col_base + c * 16 + c16;
      if (col < a.n) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = row_base + r * 16 + M::out_row(q, i);
          if (row < a.l) out[row + col * a.ldo] = acc[r][c][i];
        }
      }
    }
  }
}

// Fast path (aligned operands, every K-range a whole number of BK stages):
// the same tiling, software-pipelined -- while stage s is multiplied, the
// Omega vectors and A fragments of stage s+1 are already in flight into
// registers; staging has no per-element branches.
template <typename TE, int RT>
__global__ __launch_bounds__(256) void sketch_fast_kernel(SketchArgs<TE> a) {
  using M = MT<TE>;
  using AccV = typename M::AccV;
  constexpr int VEC = M::VEC;
  constexpr int BK = M::BK;
  constexpr int CT = M::CT;
  constexpr int SUB = BK / (4 * VEC);
  constexpr int EPV = 16 / (int)sizeof(TE);     // elements per 16-byte vector
  constexpr int VPR = BK / EPV;                 // vectors per LDS row
  constexpr int ROWS = 16 * RT;
  constexpr int NV = (ROWS * VPR + 255) / 256;  // Omega vectors per thread per stage
  constexpr int LROW = BK + 16 / (int)sizeof(TE) * 2;

  __shared__ __attribute__((aligned(16))) TE lds[ROWS * LROW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int q = lane >> 4;
  const int c16 = lane & 15;
  const int bid = blockIdx.x;
  const int split_id = bid % a.split;
  const int rest = bid / a.split;
  const int64_t ncolstrips = (a.n + 4 * CT * 16 - 1) / (4 * CT * 16);
  const int strip = (int)(rest % ncolstrips);
  const int lchunk = (int)(rest / ncolstrips);
  const int row_base = lchunk * ROWS;
  const int64_t kbeg = (int64_t)split_id * a.kchunk;
  const int64_t kend = min(a.m, kbeg + a.kchunk);
  const int nst = (int)((kend - kbeg) / BK);
  const int64_t col_base = (int64_t)strip * (4 * CT * 16) + wid * (CT * 16);

  // per-thread Omega vector slots: (row, k-offset) and validity (rows past
  // l are staged as zeros)
  const TE* optr[NV];
  int lofs[NV];
  bool oval[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int idx = tid + 256 * v;
    const int r = idx / VPR;
    const int kk = (idx % VPR) * EPV;
    const int grow = row_base + r;
    oval[v] = (idx < ROWS * VPR) && (grow < a.l);
    optr[v] = a.Pt + (int64_t)(oval[v] ? grow : 0) * a.ldp + kbeg + kk;
    lofs[v] = (idx < ROWS * VPR) ? r * LROW + kk : -1;
  }
  // per-lane A column pointers (columns past n read column 0 and are dropped)
  const TE* aptr[CT];
  bool cval[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int64_t col = col_base + c * 16 + c16;
    cval[c] = col < a.n;
    aptr[c] = a.A + (cval[c] ? col : 0) * a.lda + kbeg + q * VEC;
  }

  AccV acc[RT][CT];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = AccV{};

  uint4 ov[NV];
  Frag<TE> bf[SUB][CT];
  auto fetch = [&](int st) {
    const int64_t ko = (int64_t)st * BK;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      ov[v] = oval[v] ? *reinterpret_cast<const uint4*>(optr[v] + ko) : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub)
#pragma unroll
      for (int c = 0; c < CT; ++c) load_frag(bf[sub][c], aptr[c] + ko + sub * 4 * VEC);
  };

  if (nst > 0) fetch(0);
  for (int st = 0; st < nst; ++st) {
    __syncthreads();  // the previous stage's LDS reads are done
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (lofs[v] >= 0) *reinterpret_cast<uint4*>(&lds[lofs[v]]) = ov[v];
    Frag<TE> cur[SUB][CT];
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub)
#pragma unroll
      for (int c = 0; c < CT; ++c) cur[sub][c] = bf[sub][c];
    __syncthreads();
    if (st + 1 < nst) fetch(st + 1);
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub) {
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        Frag<TE> af;
        load_frag(af, &lds[(r * 16 + c16) * LROW + sub * 4 * VEC + q * VEC]);
#pragma unroll
        for (int s = 0; s < VEC / M::KMFMA; ++s)
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[r][c] = mfma_step<TE>(af, cur[sub][c], s, acc[r][c]);
      }
    }
  }

  typename M::Acc* out = a.out + (int64_t)split_id * a.out_split_stride;
#pragma unroll
  for (int r = 0; r < RT; ++r) {
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int64_t col = col_base + c * 16 + c16;
      if (cval[c]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = row_base + r * 16 + M::out_row(q, i);
          if (row < a.l) out[row + col * a.ldo] = acc[r][c][i];
        }
      }
    }
  }
}

// Streaming kernel (gfx950): the k-slot permutation of the kernels above,
// with the operand traffic arranged for the hardware.
//  * Workgroup tile: 32 RTW rows x 32 CTW columns of X, one K-range.  The
//    four waves form a 2 x 2 grid; each multiplies RTW row tiles by CTW
//    column tiles (16 x 16 each), so an operand fragment read from LDS feeds
//    CTW (Omega) or RTW (A) MFMAs.
//  * A stage is 128 bytes of K per row of Omega and per column of A (64
//    BF16, 128 FP8 or 32 FP32 values).
//  * Both operands go from global memory straight into LDS: buffer loads
//    with the LDS bit, 16 bytes per lane, 32-bit offsets from a wave-uniform
//    descriptor, no registers.  A direct load fills 8 rows (columns of A) of
//    a stage, lane -> (row + lane / 8, slot lane % 8); within a row the
//    16-byte slots are XOR-swizzled by (row & 7), so the MFMA operand reads
//    (16 rows at one logical slot) spread over the LDS banks.
//  * The Omega descriptor's range is its l rows (rows past l read as zeros);
//    A columns past n are clamped to column 0 (their outputs are dropped).
//  * Three stage slots rotate; the loads of stage s+2 are issued while stage
//    s multiplies, a few at a time between its MFMAs, so HBM streams during
//    the MFMAs.  The slot refilled at stage s was read at stage s-1, which
//    the barrier at the top of stage s retires.  Each slot is its own LDS
//    object, so the compiler can see that a direct load into one does not
//    feed the reads of another, and one explicit wait per stage (the loads of
//    stage s done, those of s+1 still in flight) hands the stage over.
//  * Stages past the K-range (at most two, to fill the last rotation) use
//    empty descriptors: they load zeros, touch no memory and add nothing.
//  * AT (BF16 only): the contraction runs along the columns of A instead of
//    its rows, i.e. the output is Omega A^T (l x m) for a column-major m x n
//    A, with Pt = Omega^T (n x l).  A stage of A is then 64 columns x 128
//    rows, copied as it lies in memory (256-byte LDS rows, one per column,
//    32-byte chunks XOR-swizzled by the column), and the B operand (8
//    consecutive columns of one row per lane) is read with the LDS transpose
//    read: within each 16-lane group, lane s reads 4 consecutive rows of one
//    column (column s / 4, rows 4 (s % 4) ..), and lane t receives element
//    t % 4 of lanes t / 4 + 4 e, e = 0..3 -- row t of the tile at 4
//    consecutive columns.  Rows of A past m read whatever lies there (only
//    their own, dropped, outputs see it) or zeros past the matrix's last
//    element (the descriptor's range ends there).
typedef __attribute__((address_space(3))) void lds_void_t;
typedef short v4s16 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4s16 lds_v4s16_t;

// 32-byte chunk swizzle of the transposed A stage: column kr of the stage
// stores logical chunk c at chunk c ^ at_swz(kr).  The 16 columns that one
// transpose read touches (kr = 8 g + 4 h + 0..3, g = 0..3) map to 8 distinct
// chunks.
__device__ __forceinline__ int at_swz(int kr) { return (kr & 7) ^ (((kr >> 3) & 1) << 2); }

// raw buffer descriptor word 3 for gfx9-family loads (32-bit data format)
constexpr int BUF_WORD3 = 0x00020000;

template <typename TE, int RTW, int CTW, bool RESID, bool AT = false>
__global__ __launch_bounds__(256, 1) void sketch_stream_kernel(SketchArgs<TE> a) {
  using M = MT<TE>;
  using AccV = typename M::AccV;
  using Acc = typename M::Acc;
  constexpr int VEC = M::VEC;
  constexpr int VB = VEC * (int)sizeof(TE);   // bytes of one lane operand
  constexpr int NP = VB / 16;                 // 16-byte pieces per operand
  constexpr int SB = 128;                     // stage bytes per row (8 slots)
  constexpr int BKS = SB / (int)sizeof(TE);   // K per stage
  constexpr int SUB = SB / (4 * VB);          // operand k-steps per stage
  constexpr int OROWS = 32 * RTW;             // Omega rows of the workgroup
  constexpr int ACOLS = 32 * CTW;             // A columns of the workgroup
  constexpr int NIO = OROWS / 32;             // Omega direct loads per wave per stage
  constexpr int NIA = ACOLS / 32;             // A direct loads per wave per stage
  constexpr int NI = NIO + NIA;
  constexpr int OBYTES = OROWS * SB, ABYTES = ACOLS * SB;
  constexpr int KMF = VEC / M::KMFMA;         // MFMAs per operand pair
  constexpr int IPS = (NI + SUB - 1) / SUB;   // direct loads slotted into each k-step
  static_assert(SUB >= 1 && 4 * VB * SUB == SB, "stage must hold whole operand k-steps");
  static_assert(NI <= 63, "vmcnt immediate of the hand-over");
  static_assert(!AT || (sizeof(TE) == 2 && !RESID && ACOLS == 128), "transposed A: BF16, 128 rows");

  __shared__ __attribute__((aligned(1024))) char o0[OBYTES];
  __shared__ __attribute__((aligned(1024))) char o1[OBYTES];
  __shared__ __attribute__((aligned(1024))) char o2[OBYTES];
  __shared__ __attribute__((aligned(1024))) char b0[ABYTES];
  __shared__ __attribute__((aligned(1024))) char b1[ABYTES];
  __shared__ __attribute__((aligned(1024))) char b2[ABYTES];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wr = wid & 1, wc = wid >> 1;  // this wave's row half and column half
  const int q = lane >> 4;
  const int c16 = lane & 15;
  const int bid = blockIdx.x;
  const int split_id = bid % a.split;
  const int rest = bid / a.split;
  const int64_t ncolstrips = (a.n + ACOLS - 1) / ACOLS;
  const int strip = (int)(rest % ncolstrips);
  const int lchunk = (int)(rest / ncolstrips);
  const int row_base = lchunk * OROWS;
  // K-range of this split: an even share of the stages
  const int64_t s0 = (int64_t)split_id * a.kpairs / a.split;
  const int64_t s1 = (int64_t)(split_id + 1) * a.kpairs / a.split;
  const int64_t kbeg = s0 * BKS;
  const int nst = (int)(s1 - s0);
  const int64_t col0 = (int64_t)strip * ACOLS;

  // direct-load lane offsets: row (column) 8 (w + 4 i) + lane / 8 of the
  // stage, slot (lane % 8) ^ (row & 7)
  const int swz_st = (lane & 7) ^ (lane >> 3);
  const char* obase = reinterpret_cast<const char*>(a.Pt + kbeg);
  const uint32_t orange = (uint32_t)((int64_t)a.l * a.ldp * (int64_t)sizeof(TE));
  const uint32_t orow = (uint32_t)(a.ldp * (int64_t)sizeof(TE));
  const uint32_t ooff0 = (uint32_t)(row_base + 8 * wid + (lane >> 3)) * orow + (uint32_t)(swz_st * 16);
  const char* abase = reinterpret_cast<const char*>(AT ? a.A + kbeg * a.lda : a.A + kbeg);
  const uint32_t arange = (uint32_t)(a.n * a.lda * (int64_t)sizeof(TE));
  const uint32_t acol = (uint32_t)(a.lda * (int64_t)sizeof(TE));
  // AT: bytes from the start of a stage to the end of A's last element,
  // minus those of the stages before it (clamped to the 32-bit range)
  const int64_t at_end = ((a.m - kbeg - 1) * a.lda + a.n) * (int64_t)sizeof(TE);
  const int64_t at_step = (int64_t)BKS * a.lda * (int64_t)sizeof(TE);
  uint32_t aoffs[NIA];
#pragma unroll
  for (int i = 0; i < NIA; ++i) {
    if constexpr (AT) {
      // load i of this wave fills stage columns kr = 4 (w + 4 i) .. +4; lane
      // -> (column kr + lane / 16, 16-byte slot lane % 16)
      const int kr = 4 * (wid + 4 * i) + (lane >> 4);
      const int slot = lane & 15;
      const int chunk = (slot >> 1) ^ at_swz(kr);
      aoffs[i] = (uint32_t)kr * acol + (uint32_t)((col0 + chunk * 16 + (slot & 1) * 8) * (int64_t)sizeof(TE));
    } else {
      int64_t col = col0 + 8 * (wid + 4 * i) + (lane >> 3);
      if (col >= a.n) col = 0;
      aoffs[i] = (uint32_t)col * acol + (uint32_t)(swz_st * 16);
    }
  }

  AccV acc[RTW][CTW];
#pragma unroll
  for (int r = 0; r < RTW; ++r)
#pragma unroll
    for (int c = 0; c < CTW; ++c) acc[r][c] = AccV{};

  // Residual: this lane's values of R (4 consecutive rows of one column per
  // tile) are requested now and land while the product is formed.
  uint2 rpre[RESID ? RTW : 1][RESID ? CTW : 1];
  if constexpr (RESID) {
#pragma unroll
    for (int r = 0; r < RTW; ++r)
#pragma unroll
      for (int c = 0; c < CTW; ++c) {
        const int64_t col = col0 + (wc * CTW + c) * 16 + c16;
        const int row = row_base + (wr * RTW + r) * 16 + 4 * q;
        rpre[r][c] = make_uint2(0u, 0u);
        if (a.vec_r && col < a.n && row + 3 < a.l)
          rpre[r][c] = *reinterpret_cast<const uint2*>(a.R + row + col * a.ldr);
      }
  }

  // descriptors of stage st (empty past the K-range)
  auto orsrc = [&](int st) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(obase + (int64_t)st * SB), (short)0,
                                             st < nst ? (int)orange : 0, BUF_WORD3);
  };
  auto arsrc = [&](int st) {
    if constexpr (AT) {
      int64_t rg = at_end - (int64_t)st * at_step;
      if (rg > 0x7fffffff) rg = 0x7fffffff;
      return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(abase + (int64_t)st * at_step), (short)0,
                                               st < nst ? (int)rg : 0, BUF_WORD3);
    } else {
      return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(abase + (int64_t)st * SB), (short)0,
                                               st < nst ? (int)arange : 0, BUF_WORD3);
    }
  };
  // direct load j (0 .. NI-1) of a stage: Omega loads first, then A
  auto dma = [&](__amdgpu_buffer_rsrc_t ors, __amdgpu_buffer_rsrc_t ars, char* ob, char* ab, int j) {
    if (j < NIO)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ors, (lds_void_t*)(ob + 8 * (wid + 4 * j) * SB), 16,
                                               (int)(ooff0 + (uint32_t)(32 * j) * orow), 0, 0, 0);
    else
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ars, (lds_void_t*)(ab + 8 * (wid + 4 * (j - NIO)) * SB),
                                               16, (int)aoffs[j - NIO], 0, 0, 0);
    // (AT: load j - NIO fills 1 KB = stage columns 4 (w + 4 i) .. +4, the
    // same LDS bytes as 8 rows of 128 bytes)
  };
  auto load_stage = [&](int st, char* ob, char* ab) {
    const auto ors = orsrc(st);
    const auto ars = arsrc(st);
#pragma unroll
    for (int j = 0; j < NI; ++j) dma(ors, ars, ob, ab, j);
  };

  // operand reads: row (column) c16 of a 16-row tile; logical slot of (sub,
  // piece p) = sub*4*NP + q*NP + p, stored at slot ^ (c16 & 7)
  const int o_rd = (wr * RTW * 16 + c16) * SB;
  const int a_rd = (wc * CTW * 16 + c16) * SB;
  const int swz = c16 & 7;
  // Stage st: MFMAs from (ob, ab); the loads of stage st + 2 go to (nob, nab),
  // spread over the k-steps.
  auto stage = [&](int st, const char* ob, const char* ab, char* nob, char* nab) {
    const auto ors = orsrc(st + 2);
    const auto ars = arsrc(st + 2);
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub) {
      Frag<TE> af[RTW], bf[CTW];
      if constexpr (AT) {
        // columns sub*32 + 8 q + 4 h + (c16 / 4) of the stage, rows
        // 4 (c16 % 4) .. +4 of tile c
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int kr = sub * 32 + 8 * q + 4 * h + (c16 >> 2);
          const int sw = at_swz(kr);
#pragma unroll
          for (int c = 0; c < CTW; ++c) {
            const int chunk = (wc * CTW + c) ^ sw;
            const v4s16 t = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                (lds_v4s16_t*)(ab + kr * 256 + chunk * 32 + 8 * (c16 & 3)));
            __builtin_memcpy(reinterpret_cast<char*>(bf[c].v) + 8 * h, &t, 8);
          }
        }
      }
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int slot = (sub * 4 * NP + q * NP + p) ^ swz;
#pragma unroll
        for (int c = 0; c < CTW; ++c)
          if constexpr (!AT)
            reinterpret_cast<uint4*>(bf[c].v)[p] =
                *reinterpret_cast<const uint4*>(ab + a_rd + c * 16 * SB + slot * 16);
#pragma unroll
        for (int r = 0; r < RTW; ++r)
          reinterpret_cast<uint4*>(af[r].v)[p] =
              *reinterpret_cast<const uint4*>(ob + o_rd + r * 16 * SB + slot * 16);
      }
#pragma unroll
      for (int j = 0; j < IPS; ++j)
        if (sub * IPS + j < NI) dma(ors, ars, nob, nab, sub * IPS + j);
#pragma unroll
      for (int r = 0; r < RTW; ++r)
#pragma unroll
        for (int s = 0; s < KMF; ++s)
#pragma unroll
          for (int c = 0; c < CTW; ++c) acc[r][c] = mfma_step<TE>(af[r], bf[c], s, acc[r][c]);
      // issue order: this k-step's LDS reads, then its MFMAs with the loads
      // of stage st + 2 slotted in between
      constexpr int NM = RTW * CTW * KMF;
      constexpr int GAP = NM / (IPS + 1) > 0 ? NM / (IPS + 1) : 1;
      __builtin_amdgcn_sched_group_barrier(0x100, RTW * NP + (AT ? 2 * CTW : CTW * NP), 0);
#pragma unroll
      for (int v = 0; v < IPS; ++v) {
        __builtin_amdgcn_sched_group_barrier(0x008, GAP, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, NM - IPS * GAP, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  // Stage hand-over: this wave's direct loads of stage st are done (those of
  // st+1, NI of them, may still be in flight), then a barrier.  This is not
  // __syncthreads(): its workgroup fence would also wait for the loads of
  // st+1.  The statement loads nothing; its memory clobber keeps the
  // compiler from moving LDS accesses across it.
  auto handover = [&]() { asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(NI) : "memory"); };
  load_stage(0, o0, b0);
  load_stage(1, o1, b1);
  for (int st = 0; st < nst; st += 3) {
    handover();
    stage(st, o0, b0, o2, b2);
    handover();
    stage(st + 1, o1, b1, o0, b0);
    handover();
    stage(st + 2, o2, b2, o1, b1);
  }
  // drain the direct loads of the stages past the end (empty descriptors)
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

  if constexpr (RESID) {
    // ||R - product||^2 and ||R||^2 over this tile, in FP64; lane (c16, q)
    // holds rows 16 t + 4 q .. +4 of column c16 of tile (t, c)
    double sd = 0.0, sa = 0.0;
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
#pragma unroll
      for (int c = 0; c < CTW; ++c) {
        const int64_t col = col0 + (wc * CTW + c) * 16 + c16;
        const int row = row_base + (wr * RTW + r) * 16 + 4 * q;
        if (col >= a.n || row >= a.l) continue;
        const uint16_t* p = a.R + row + col * a.ldr;
        uint16_t rb[4];
        if (a.vec_r && row + 3 < a.l) {
          __builtin_memcpy(rb, &rpre[r][c], 8);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) rb[i] = (row + i < a.l) ? p[i] : (uint16_t)0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double rv = (double)__uint_as_float((uint32_t)rb[i] << 16);
          const double d = rv - (double)acc[r][c][i];
          sd = fma(d, d, sd);
          sa = fma(rv, rv, sa);
        }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      sd += __shfl_xor(sd, off, 64);
      sa += __shfl_xor(sa, off, 64);
    }
    __shared__ double red[2][4];
    if (lane == 0) {
      red[0][wid] = sd;
      red[1][wid] = sa;
    }
    __syncthreads();
    if (tid == 0) {
      a.partials[2 * (int64_t)bid] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
      a.partials[2 * (int64_t)bid + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
    return;
  } else {
    // Write the tile (X or this split's partial): lane (c16, q) holds rows
    // 16 t + 4 q .. +4 of column c16 of tile (t, c), 4 consecutive values of
    // one column.
    Acc* out = a.out + (int64_t)split_id * a.out_split_stride;
#pragma unroll
    for (int r = 0; r < RTW; ++r) {
#pragma unroll
      for (int c = 0; c < CTW; ++c) {
        const int64_t col = col0 + (wc * CTW + c) * 16 + c16;
        const int row = row_base + (wr * RTW + r) * 16 + 4 * q;
        if (col >= a.n || row >= a.l) continue;
        Acc* p = out + row + col * a.ldo;
        if (a.vec_out && row + 3 < a.l) {
          *reinterpret_cast<AccV*>(p) = acc[r][c];
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (row + i < a.l) p[i] = acc[r][c][i];
        }
      }
    }
  }
}

// X(r, j) = sum_s part[s](r, j) in a fixed order, converted to the X type.
template <typename TA, typename TX>
__global__ void split_reduce_kernel(const TA* part, int split, int64_t stride, int64_t l,
                                    int64_t n, int64_t ldp, TX* X, int64_t ldx) {
  const int64_t total = l * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % l, j = e / l;
    const int64_t o = r + j * ldp;
    TA s = part[o];
    // eight loads in flight per round, added in the same order as one by one
    int t = 1;
    for (; t + 8 <= split; t += 8) {
      TA v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(t + u) * stride + o];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; t < split; ++t) s += part[(int64_t)t * stride + o];
    X[r + j * ldx] = (TX)s;
  }
}

// One launch with RT row tiles per l-chunk; the fast kernel needs aligned
// operands and whole BK stages in every K-range.
template <typename TE, int RT>
static void launch_rt(rpid_ctx ctx, const SketchArgs<TE>& a, int64_t grid, bool aligned, bool fast) {
  if (fast)
    hipLaunchKernelGGL((sketch_fast_kernel<TE, RT>), dim3((unsigned)grid), dim3(256), 0, ctx->stream,
                       a);
  else if (aligned)
    hipLaunchKernelGGL((sketch_kernel<TE, RT, true>), dim3((unsigned)grid), dim3(256), 0,
                       ctx->stream, a);
  else
    hipLaunchKernelGGL((sketch_kernel<TE, RT, false>), dim3((unsigned)grid), dim3(256), 0,
                       ctx->stream, a);
}

// Row tiles are a compile-time count (the MFMA loop is then straight-line
// code that the compiler can software-pipeline); a chunk of `need` tiles runs
// the smallest instantiated count >= need, with the extra rows discarded.
template <typename TE>
static int rows_per_chunk(int need) {
  static constexpr int counts[] = {1, 2, 3, 4, 5, 6, 8, 10, 13, 17};
  for (int c : counts)
    if (need <= c) return c;
  return 0;
}

template <typename TE>
static void launch_sketch(rpid_ctx ctx, const SketchArgs<TE>& a, int64_t grid, bool aligned,
                          bool fast, int rt) {
  switch (rt) {
    case 1: launch_rt<TE, 1>(ctx, a, grid, aligned, fast); break;
    case 2: launch_rt<TE, 2>(ctx, a, grid, aligned, fast); break;
    case 3: launch_rt<TE, 3>(ctx, a, grid, aligned, fast); break;
    case 4: launch_rt<TE, 4>(ctx, a, grid, aligned, fast); break;
    case 5: launch_rt<TE, 5>(ctx, a, grid, aligned, fast); break;
    case 6: launch_rt<TE, 6>(ctx, a, grid, aligned, fast); break;
    case 8: launch_rt<TE, 8>(ctx, a, grid, aligned, fast); break;
    case 10: launch_rt<TE, 10>(ctx, a, grid, aligned, fast); break;
    case 13: launch_rt<TE, 13>(ctx, a, grid, aligned, fast); break;
    default: launch_rt<TE, 17>(ctx, a, grid, aligned, fast); break;
  }
}

template <typename TE, int CTW, bool AT = false>
static void launch_stream(rpid_ctx ctx, const SketchArgs<TE>& a, int64_t grid, int rtw) {
  switch (rtw) {
#define RPID_STREAM_RTW(R)                                                                  \
  case R:                                                                                  \
    hipLaunchKernelGGL((sketch_stream_kernel<TE, R, CTW, false, AT>), dim3((unsigned)grid), dim3(256), 0, \
                       ctx->stream, a);                                                    \
    break;
    RPID_STREAM_RTW(1)
    RPID_STREAM_RTW(2)
    RPID_STREAM_RTW(3)
    RPID_STREAM_RTW(4)
    RPID_STREAM_RTW(5)
    RPID_STREAM_RTW(6)
    RPID_STREAM_RTW(7)
    RPID_STREAM_RTW(8)
    default:
      RPID_STREAM_RTW(9)
#undef RPID_STREAM_RTW
  }
}

// Column tiles per wave of the streaming kernel, per element type.
template <typename TE>
struct StreamCTW {
  static constexpr int value = 4;
};

// The streaming kernel (BF16, FP8, FP32 operands): aligned operands, K a
// whole number of 128-byte stages, 32-bit operand offsets.  Returns false if
// it does not apply.  AT (BF16): the product is Pt^T A^T for a column-major
// A of `n` rows and `m` columns (K = m runs along its columns); the output
// is l x n as always.  `max_split` caps the split-K count.
template <typename TE, bool AT = false>
static bool sketch_stream(rpid_ctx ctx, const TE* Pt, int64_t ldp, const TE* A, int64_t lda,
                          int64_t m, int64_t n, int64_t l, typename MT<TE>::Acc* X, int64_t ldx,
                          size_t ws_off, int* err, int64_t max_split = 16) {
  using Acc = typename MT<TE>::Acc;
  constexpr int CTW = StreamCTW<TE>::value;
  constexpr int BKS = 128 / (int)sizeof(TE);
  constexpr int RTWMAX = 9;  // up to 288 rows per l-chunk
  const int64_t sz = (int64_t)sizeof(TE);
  const bool aligned = ((uintptr_t)A % 16 == 0) && ((uintptr_t)Pt % 16 == 0) && (lda * sz) % 16 == 0 &&
                       (ldp * sz) % 16 == 0;
  if (!aligned || m % BKS != 0) return false;
  if (AT) {
    // 16-byte pieces never straddle the last row; in-stage offsets fit 32 bits
    if (n % 8 != 0 || lda < n || (int64_t)BKS * lda * sz + n * sz >= ((int64_t)1 << 31)) return false;
  } else if (n * lda * sz >= ((int64_t)1 << 31)) {
    return false;
  }
  if (l * ldp * sz >= ((int64_t)1 << 31)) return false;
  // l-chunks of at most 2 RTWMAX row tiles, as even as the tile count allows
  const int ltiles = (int)((l + 15) / 16);
  const int lchunks = (ltiles + 2 * RTWMAX - 1) / (2 * RTWMAX);
  const int rtw = ((ltiles + lchunks - 1) / lchunks + 1) / 2;
  const int64_t strips = (n + 32 * CTW - 1) / (32 * CTW);
  const int64_t kst = m / BKS;  // stages
  int64_t split = (int64_t)ctx->num_cu / (strips * lchunks);
  if (split > kst) split = kst;
  if (split > max_split) split = max_split;
  if (split < 1) split = 1;
  SketchArgs<TE> a{};
  a.Pt = Pt;
  a.ldp = ldp;
  a.A = A;
  a.lda = lda;
  a.m = m;
  a.n = n;
  a.l = (int)l;
  a.split = (int)split;
  a.kchunk = 0;
  a.ltiles = ltiles;
  a.kpairs = kst;
  if (split == 1) {
    a.out = X;
    a.ldo = ldx;
    a.out_split_stride = 0;
    a.vec_out = ((uintptr_t)X % 16 == 0) && (ldx % 4 == 0);
  } else {
    Carve cv;
    cv.off = ws_off;
    size_t o_part = cv.take<Acc>((size_t)split * l * n);
    *err = ws_check(ctx, cv.off);
    if (*err != RPID_OK) return true;
    a.out = ws_ptr<Acc>(ctx, o_part);
    a.ldo = l;
    a.out_split_stride = l * n;
    a.vec_out = (l % 4 == 0);
  }
  launch_stream<TE, CTW, AT>(ctx, a, split * strips * lchunks, rtw);
  *err = hipGetLastError() == hipSuccess ? RPID_OK : RPID_ERR_HIP;
  if (*err == RPID_OK && split > 1) {
    int64_t blocks = (l * n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((split_reduce_kernel<Acc, Acc>), dim3((unsigned)blocks), dim3(256), 0,
                       ctx->stream, a.out, (int)split, l * n, l, n, l, X, ldx);
    *err = hipGetLastError() == hipSuccess ? RPID_OK : RPID_ERR_HIP;
  }
  return true;
}

// ||R - P Q||_F^2 and ||R||_F^2 on the streaming kernel (BF16 operands, FP32
// accumulation, FP64 epilogue): Pt is r x m and Q is r x n, both
// k-contiguous; 256 x 128 tiles, one per workgroup, partial sums per
// workgroup in launch order.  Returns false (nothing launched) if the shapes
// or alignments do not suit it; otherwise *count is the number of partials.
bool residual_stream_bf16(rpid_ctx ctx, int64_t m, int64_t n, int64_t r, const uint16_t* R,
                          int64_t ldr, const uint16_t* Pt, int64_t ldpt, const uint16_t* Q,
                          int64_t ldq, double* partials, int64_t* count, int* err) {
  constexpr int RTW = 8, CTW = 4, BKS = 64;
  const bool aligned = ((uintptr_t)Pt % 16 == 0) && ((uintptr_t)Q % 16 == 0) && (ldpt * 2) % 16 == 0 &&
                       (ldq * 2) % 16 == 0;
  if (!aligned || r % BKS != 0 || r < BKS) return false;
  if (n * ldq * 2 >= ((int64_t)1 << 31) || m * ldpt * 2 >= ((int64_t)1 << 31)) return false;
  const int64_t lchunks = (m + 32 * RTW - 1) / (32 * RTW);
  const int64_t strips = (n + 32 * CTW - 1) / (32 * CTW);
  SketchArgs<uint16_t> a{};
  a.Pt = Pt;
  a.ldp = ldpt;
  a.A = Q;
  a.lda = ldq;
  a.m = r;
  a.n = n;
  a.l = (int)m;
  a.split = 1;
  a.kchunk = 0;
  a.ltiles = (int)((m + 15) / 16);
  a.kpairs = r / BKS;
  a.R = R;
  a.ldr = ldr;
  a.vec_r = ((uintptr_t)R % 8 == 0) && (ldr % 4 == 0);
  a.partials = partials;
  const int64_t grid = lchunks * strips;
  hipLaunchKernelGGL((sketch_stream_kernel<uint16_t, RTW, CTW, true>), dim3((unsigned)grid), dim3(256),
                     0, ctx->stream, a);
  *err = hipGetLastError() == hipSuccess ? RPID_OK : RPID_ERR_HIP;
  *count = grid;
  return true;
}

template <typename TE>
static int sketch_impl(rpid_ctx ctx, const TE* Pt, int64_t ldp, const TE* A, int64_t lda,
                       int64_t m, int64_t n, int64_t l, typename MT<TE>::Acc* X, int64_t ldx,
                       size_t ws_off, int64_t max_split) {
  using M = MT<TE>;
  using Acc = typename M::Acc;
  constexpr int RTMAX = 17;  // up to 272 rows per l-chunk
  if (l < 1 || l > 1024 || m < 1 || n < 1) return RPID_ERR_UNSUPPORTED;
  const int ltiles = (int)((l + 15) / 16);
  const int lchunks = (ltiles + RTMAX - 1) / RTMAX;
  const int rt = rows_per_chunk<TE>((ltiles + lchunks - 1) / lchunks);
  const int64_t colw = 4 * M::CT * 16;
  const int64_t strips = (n + colw - 1) / colw;
  // Split K so that the grid fills the chip in one round (one workgroup per
  // CU: the tile holds 204+ accumulator registers per lane).
  const int64_t base_wgs = strips * lchunks;
  int64_t split = (int64_t)ctx->num_cu / base_wgs;
  const int64_t kblocks = (m + M::BK - 1) / M::BK;
  if (split > kblocks) split = kblocks;
  if (split > max_split) split = max_split;
  if (split < 1) split = 1;
  int64_t kchunk = ((kblocks + split - 1) / split) * M::BK;
  split = (m + kchunk - 1) / kchunk;

  const bool aligned = ((uintptr_t)A % 16 == 0) && ((uintptr_t)Pt % 16 == 0) &&
                       (lda * (int64_t)sizeof(TE)) % 16 == 0 &&
                       (ldp * (int64_t)sizeof(TE)) % 16 == 0;

  SketchArgs<TE> a;
  a.Pt = Pt;
  a.ldp = ldp;
  a.A = A;
  a.lda = lda;
  a.m = m;
  a.n = n;
  a.l = (int)l;
  a.split = (int)split;
  a.kchunk = kchunk;
  a.ltiles = ltiles;
  if (split == 1) {
    a.out = X;
    a.ldo = ldx;
    a.out_split_stride = 0;
  } else {
    Carve cv;
    cv.off = ws_off;
    size_t o_part = cv.take<Acc>((size_t)split * l * n);
    RPID_CHECK(ws_check(ctx, cv.off));
    a.out = ws_ptr<Acc>(ctx, o_part);
    a.ldo = l;
    a.out_split_stride = l * n;
  }
  const int64_t grid = split * strips * lchunks;
  launch_sketch<TE>(ctx, a, grid, aligned, aligned && m % M::BK == 0, rt);
  RPID_HIP_CHECK(hipGetLastError());
  if (split > 1) {
    int64_t blocks = (l * n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((split_reduce_kernel<Acc, Acc>), dim3((unsigned)blocks), dim3(256), 0,
                       ctx->stream, a.out, (int)split, l * n, l, n, l, X, ldx);
    RPID_HIP_CHECK(hipGetLastError());
  }
  return RPID_OK;
}

size_t sketch_workspace_bytes(rpid_ctx ctx, int64_t m, int64_t n, int64_t l, int acc_bytes) {
  (void)ctx;
  (void)m;
  return (size_t)16 * l * n * acc_bytes + 512;
}

int sketch_f64(rpid_ctx ctx, const double* Pt, int64_t ldp, const double* A, int64_t lda,
               int64_t m, int64_t n, int64_t l, double* X, int64_t ldx, size_t ws_off,
               int64_t max_split) {
  return sketch_impl<double>(ctx, Pt, ldp, A, lda, m, n, l, X, ldx, ws_off, max_split);
}
int sketch_f32(rpid_ctx ctx, const float* Pt, int64_t ldp, const float* A, int64_t lda,
               int64_t m, int64_t n, int64_t l, float* X, int64_t ldx, size_t ws_off,
               int64_t max_split) {
  int err = RPID_OK;
  if (l >= 1 && l <= 1024 &&
      sketch_stream<float>(ctx, Pt, ldp, A, lda, m, n, l, X, ldx, ws_off, &err, max_split))
    return err;
  return sketch_impl<float>(ctx, Pt, ldp, A, lda, m, n, l, X, ldx, ws_off, max_split);
}
int sketch_e4m3(rpid_ctx ctx, const uint8_t* Pt, int64_t ldp, const uint8_t* A, int64_t lda,
                int64_t m, int64_t n, int64_t l, float* X, int64_t ldx, size_t ws_off) {
  int err = RPID_OK;
  if (l >= 1 && l <= 1024 && sketch_stream<uint8_t>(ctx, Pt, ldp, A, lda, m, n, l, X, ldx, ws_off, &err))
    return err;
  return sketch_impl<uint8_t>(ctx, Pt, ldp, A, lda, m, n, l, X, ldx, ws_off, 16);
}
int sketch_bf16(rpid_ctx ctx, const uint16_t* Pt, int64_t ldp, const uint16_t* A, int64_t lda,
                int64_t m, int64_t n, int64_t l, float* X, int64_t ldx, size_t ws_off,
                int64_t max_split) {
  int err = RPID_OK;
  if (l >= 1 && l <= 1024 &&
      sketch_stream<uint16_t>(ctx, Pt, ldp, A, lda, m, n, l, X, ldx, ws_off, &err, max_split))
    return err;
  return sketch_impl<uint16_t>(ctx, Pt, ldp, A, lda, m, n, l, X, ldx, ws_off, max_split);
}

// Y^T = Omega A^T (l x m) for a column-major m x n BF16 A, with Ot = Omega^T
// (n x l, BF16): the streaming kernel with K along the columns of A, so A is
// read in place.  RPID_ERR_UNSUPPORTED (nothing launched) when the shapes or
// alignments do not suit it (n a multiple of 64, m of 8, 16-byte aligned
// operands and leading dimensions).
int sketch_at_bf16(rpid_ctx ctx, const uint16_t* Ot, int64_t ldot, const uint16_t* A, int64_t lda,
                   int64_t m, int64_t n, int64_t l, float* Yt, int64_t ldyt, size_t ws_off) {
  int err = RPID_OK;
  if (l < 1 || l > 1024 || m < 1 || n < 1) return RPID_ERR_UNSUPPORTED;
  if (!sketch_stream<uint16_t, true>(ctx, Ot, ldot, A, lda, n, m, l, Yt, ldyt, ws_off, &err))
    return RPID_ERR_UNSUPPORTED;
  return err;
}

}  // namespace rpid
