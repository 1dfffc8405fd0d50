/*
 * rpid.h -- C-ABI of the MI355X (gfx950) library for randomized LUPP skeleton
 * selection: interpolative (ID) and CUR decompositions.
 *
 * Method: Dong & Martinsson, "Simpler is better: a comparative study of
 * randomized pivoting algorithms for CUR and interpolative decompositions",
 * Alg. 2 (Randomized LUPP skeleton selection) with the sketch-based ID
 * coefficients of Sec. 4 and the stable CUR construction of the Remark
 * "Stable CUR" (eq. cur_stable).
 *
 * Conventions (all entry points):
 *  - Matrices are DEVICE pointers, column-major, with a leading dimension
 *    ld >= number of rows.  Element type is given by an rpid_dtype argument.
 *  - Index vectors (J_s, I_s) are DEVICE int64 arrays, 0-based, in pivot
 *    order (the paper's MATLAB indices are 1-based).
 *  - Host scalars (k_eff, eta, rel_fro) are HOST pointers; a call that
 *    receives a non-NULL host scalar synchronises the context's stream
 *    before returning.  Calls with no host scalar only enqueue work.
 *  - The caller allocates and owns every input and output buffer.  The
 *    context owns a device workspace, grown on demand (hipMalloc) and freed
 *    by rpid_destroy.  No pointer passed in is retained after a call.
 *  - All work is enqueued on the context's HIP stream.  A context is used by
 *    one host thread at a time.
 *  - Return value: RPID_OK (0); a negative value -i when the i-th argument
 *    (1-based, the context counting as argument 1) is invalid; one of the
 *    RPID_ERR_* codes; or a positive value t+1 when the pivot of 0-based
 *    step t is exactly zero (rank deficiency, the premise of Lemma 1
 *    violated), in which case *k_eff = t and only the first t pivots are
 *    defined (LAPACK getrf "info" convention).
 */
#ifndef RPID_H
#define RPID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RPID_F64 = 0,      /* IEEE binary64 */
  RPID_F32 = 1,      /* IEEE binary32 */
  RPID_BF16 = 2,     /* bfloat16 (8-bit exponent, 7-bit mantissa) */
  RPID_FP8_E4M3 = 3  /* OCP FP8 E4M3 (max 448, no infinities) */
} rpid_dtype;

typedef enum {
  RPID_RESIDUAL_ID = 0,    /* column ID  A ~ A(:, J) Z               */
  RPID_RESIDUAL_CUR = 1,   /* CUR        A ~ A(:, J) U A(I, :)       */
  RPID_RESIDUAL_ROW_ID = 2 /* row ID     A ~ Z^T A(I, :), Z is k x m */
} rpid_residual_kind;

#define RPID_OK 0
#define RPID_ERR_NONFINITE (-100)   /* NaN/Inf in a matrix handed to pivoting */
#define RPID_ERR_HIP (-101)         /* a HIP runtime call failed */
#define RPID_ERR_NOMEM (-102)       /* workspace allocation failed */
#define RPID_ERR_UNSUPPORTED (-103) /* dtype combination or size not supported */
#define RPID_ERR_LAUNCH (-104)      /* cooperative launch could not co-schedule the grid */
#define RPID_ERR_TIMEOUT (-105)     /* a device-side wait exceeded its spin limit */
#define RPID_ERR_BREAKDOWN (-106)   /* Cholesky breakdown while orthonormalising C or R^T */
#define RPID_ERR_SCRATCH (-107)     /* input larger than the fixed scratch of rpid_sketch_noalloc */

typedef struct rpid_ctx_s* rpid_ctx;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
int rpid_create(rpid_ctx* out, int device, void* hip_stream);
/* Free the workspace and the context (synchronises its stream first). */
int rpid_destroy(rpid_ctx ctx);
/* Change the stream later calls enqueue on. */
int rpid_set_stream(rpid_ctx ctx, void* hip_stream);
/* Static description of a status code. */
const char* rpid_status_string(int status);
/* Library ABI version (increments on any signature change). */
int rpid_version(void);

/*
 * S2 -- row sketch X = Omega A (Alg. 2, step 2; the Gaussian embedding of
 * Sec. 2.2, drawn by the caller so that any reference sees the same values).
 *   A      m x n, lda >= m, type a_t
 *   Omega  l x m, ldo >= l, type o_t
 *   X      l x n, ldx >= l, type x_t (output)
 * Supported (a_t, o_t, x_t): (F64,F64,F64) on FP64 MFMA, (F32,F32,F32) on
 * FP32 MFMA, (BF16,BF16,F32) on BF16 MFMA with FP32 accumulation.
 * 1 <= l <= 1024.
 */
int rpid_sketch(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n, int64_t lda,
                const void* Omega, rpid_dtype o_t, int64_t l, int64_t ldo, void* X, rpid_dtype x_t,
                int64_t ldx);

/*
 * rpid_sketch for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, types, kernels and result, but the call's scratch (the
 * packed Omega^T, m l e_A bytes, and the split-K partial sums) lives in a
 * fixed 64 MiB device array that the library holds on each device until the
 * process ends, instead of the context's growable workspace.  The call
 * performs no hipMalloc, hipFree or other allocation.
 * Limits: m * l * e_A + 576 bytes must fit in 64 MiB (e_A = 8, 4, 2 for
 * F64, F32, BF16), else RPID_ERR_SCRATCH before anything is enqueued; the
 * split-K count is capped so that the partial sums fit (for larger l * n
 * the summation order, and so the last bits of X, can differ from
 * rpid_sketch's; where rpid_sketch's own split fits, X is bitwise the same).
 * Every call on a device shares that device's array and leaves its contents
 * behind (nothing in it has to start at zero); two calls that overlap on one
 * device (contexts on different streams) race on it and must be ordered by
 * the caller.
 * Errors: as rpid_sketch, plus RPID_ERR_SCRATCH.
 */
int rpid_sketch_noalloc(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                        int64_t lda, const void* Omega, rpid_dtype o_t, int64_t l, int64_t ldo,
                        void* X, rpid_dtype x_t, int64_t ldx);

/*
 * Row sketch with one plain power iteration, eq. (def_power_iter) with q = 1
 * (the Rand-LUPP-1piter variant of Sec. 5): X = Omega A^T A, formed as
 * Y^T = Omega A^T and then X = Y^T A.  Omega here is l x n (it multiplies
 * the columns of A).
 *   A      m x n, lda >= m, type a_t
 *   Omega  l x n, ldo >= l, type o_t
 *   X      l x n, ldx >= l, type x_t (output)
 * Supported (a_t, o_t, x_t): (F64,F64,F64), (F32,F32,F32) and
 * (BF16,BF16,F32).  In the BF16 form Y^T is formed in FP32 and enters the
 * second product as two BF16 terms (about 16 significant bits).
 * 1 <= l <= 512.  Workspace: the Y^T factors (about 4 l (m + n) bytes, plus
 * split-K partials), and a transposed copy of A (m n e_A bytes) except in
 * the BF16 form when A is 16-byte aligned, lda a multiple of 8, n a multiple
 * of 64 and m of 8 (then A is read in place).
 * Errors: -position for an invalid argument, RPID_ERR_UNSUPPORTED for other
 * type combinations, RPID_ERR_NOMEM if the workspace cannot grow.
 */
int rpid_sketch_power1(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                       int64_t lda, const void* Omega, rpid_dtype o_t, int64_t l, int64_t ldo,
                       void* X, rpid_dtype x_t, int64_t ldx);

/*
 * Two-sided sketch of the streaming skeleton selection (Alg. 3, step 2): the
 * row sketch X = Gamma A and the column sketch Y = A Omega^T, the latter
 * returned transposed as Yt = Y^T = Omega A^T, so that the row-wise pivoting
 * of Alg. 3, step 4 is rpid_select_columns on Yt (its pivots are rows of A)
 * and the row ID coefficients are rpid_id_coeffs on Yt.
 *   A      m x n, lda >= m, type a_t
 *   Gamma  l x m, ldg >= l, type a_t (independent of Omega)
 *   Omega  l x n, ldo >= l, type a_t
 *   X      l x n, ldx >= l, type out_t (output)
 *   Yt     l x m, ldyt >= l, type out_t (output)
 * a_t F64 gives out_t F64; F32 and BF16 give out_t F32 (FP32 accumulation).
 * 1 <= l <= 1024.  BF16 with A 16-byte aligned, lda a multiple of 8, n a
 * multiple of 64 and m of 8 reads A once: row blocks of at most 128 MiB feed
 * both products back to back (the second read of a block comes from the
 * last-level cache); other cases form a transposed copy of A in the
 * workspace and read A twice.
 * Errors: -position for an invalid argument (-16: out_t does not match
 * a_t), RPID_ERR_NOMEM if the workspace cannot grow.
 */
int rpid_sketch_two_sided(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                          int64_t lda, const void* Gamma, int64_t ldg, const void* Omega,
                          int64_t ldo, int64_t l, void* X, int64_t ldx, void* Yt, int64_t ldyt,
                          rpid_dtype out_t);

/*
 * Sketch-only CUR core (the cheap form after Alg. 3): U = S^{-1} with
 * S = A(I, J) the k x k intersection of the skeletons, so that A ~ C U R
 * without another pass over A (accuracy and stability below those of the
 * stable core that rpid_cur computes).  S is factored by LU with row
 * pivoting in FP64.
 *   A   m x n, lda >= m, type a_t (F64, F32 or BF16)
 *   J   k column indices, I k row indices (device, int64, 0-based)
 *   U   k x k FP64 (device, ldu >= k, output)
 * Returns 0, or t + 1 > 0 if S has an exactly zero pivot at step t (U is
 * then not written), or -position for an invalid argument.
 */
int rpid_cur_sketch(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n, int64_t lda,
                    int64_t k, const int64_t* J, const int64_t* I, double* U, int64_t ldu);

/*
 * S2, FP8 form -- X = Omega A with A and Omega quantised to OCP E4M3 with
 * power-of-two scales, multiplied on FP8 MFMA with FP32 accumulation, and
 * the scales undone exactly in X:
 *   A_q(:, j) = e4m3(A(:, j) * 2^ea[j]),  ea[j] = floor(log2(448 / max|A(:, j)|))
 *   Om_q      = e4m3(Omega * 2^eo),       eo    = floor(log2(448 / max|Omega|))
 *   X(:, j)   = (Om_q A_q(:, j)) * 2^-(eo + ea[j])
 * (e4m3 rounds to nearest even and saturates at +-448.)  A is F32 (m x n),
 * Omega F32 (l x m), X F32 (l x n).  A column of zeros gets ea[j] = 0.
 */
int rpid_sketch_fp8(rpid_ctx ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                    const float* Omega, int64_t l, int64_t ldo, float* X, int64_t ldx);

/*
 * S3 -- column-wise LU with partial pivoting of the sketch (Alg. 2, step 3;
 * eq. def_LUPP), k steps, i.e. getrf of the n x k panel X(0:k, :)^T.
 * Step t picks the remaining column j with the largest |X^(t)(t, j)|; ties
 * go to the smallest j.  Only the first k rows of X are read (the first k
 * pivots depend on nothing else).
 *   X      l x n, ldx >= l, type x_t in {F64, F32}; the factorisation runs
 *          in x_t arithmetic
 *   k      1 <= k <= min(l, n), k <= 1024
 *   J      int64[k]   pivots in pivot order (0-based columns of X)
 *   Lf     n x k, ldl >= n, type x_t: Lf(j, t) = multiplier of column j at
 *          step t (|.| <= 1), 1 at its own pivot step, 0 after it
 *   Uf     k x k, ldu >= k, type x_t: upper triangular, Uf(t, c) = row c of
 *          the updated sketch at pivot p_t (zero below the diagonal); then
 *          X(0:k, :)^T = Lf Uf up to rounding
 *   diagU  k values of type x_t: |Uf(t, t)| (pivot magnitudes); may be NULL
 *   k_eff  host int64*, NULL to skip the synchronising status read
 * Returns RPID_ERR_NONFINITE if the panel holds NaN/Inf (nothing defined).
 */
int rpid_select_columns(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n,
                        int64_t ldx, int64_t k, int64_t* J, void* Lf, int64_t ldl, void* Uf,
                        int64_t ldu, void* diagU, int64_t* k_eff);

/*
 * S3 without a host read: rpid_select_columns (same pivots, same outputs)
 * with its status written to a device word in stream order, so that the work
 * that depends on J can be enqueued before the pivots are known.
 *   X .. diagU   as for rpid_select_columns
 *   status_dev   DEVICE int64*, caller-owned: receives 0 (k pivots), t + 1
 *                for an exactly zero pivot at 0-based step t (the first t
 *                pivots are defined), or a negative RPID_ERR_* code
 *                (RPID_ERR_NONFINITE for NaN/Inf in X, RPID_ERR_TIMEOUT if
 *                the pivot exchange gave up)
 * Returns RPID_OK once the work is enqueued, a negative argument index
 * (-14 for a NULL status_dev), or a launch error; it never synchronises.
 * When the status is not 0 the entries of J past the defined pivots are left
 * as they were.  Every call of this library that takes J or I treats entries
 * outside [0, n) (resp. [0, m)) as absent, reading zeros and writing
 * nothing, so work enqueued on such J computes garbage but never accesses
 * memory out of bounds; the caller discards it after reading the status.
 */
int rpid_select_columns_async(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n,
                              int64_t ldx, int64_t k, int64_t* J, void* Lf, int64_t ldl, void* Uf,
                              int64_t ldu, void* diagU, int64_t* status_dev);

/*
 * Sparse sign embedding (Sec. 2.2, third embedding): Gamma (l x m) has in
 * column i the entries signs[i, s] (+-1) at rows rows[i, s], s < zeta, times
 * `scale`; X = Gamma A for a dense A.  The draws are the caller's:
 *   rows   int32 m x zeta, row-major (rows[i * zeta + s]), values in [0, l),
 *          distinct within a row (an index outside [0, l) adds nothing)
 *   signs  int8 m x zeta, row-major, +1 or -1
 *   zeta   1 <= zeta <= min(l, 64); scale > 0 (the paper's 2 <= zeta <= l;
 *          its normalisation is left to the caller: pivots do not depend on it)
 *   A, a_t, m, n, lda, X, x_t, ldx, l as for rpid_sketch, (a_t, x_t) in
 *          {(F64,F64), (F32,F32), (BF16,F32)}
 * The embedding is expanded to exact +-1 entries in A's type and applied by
 * the dense MFMA sketch; the scale multiplies X afterwards.
 */
int rpid_sketch_sparse_sign(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                            int64_t lda, const int32_t* rows, const int8_t* signs, int64_t zeta,
                            int64_t l, double scale, void* X, rpid_dtype x_t, int64_t ldx);

/*
 * SRTT embedding (Sec. 2.2, second embedding) with the discrete Hartley
 * transform: Gamma = sqrt(m / l) Pi_{m->l} T Phi Pi_{m->m}, i.e.
 * Gamma(r, perm[b]) = cas(2 pi sel[r] b / m) phi[b] / sqrt(l) with cas = cos +
 * sin; X = Gamma A.  The draws are the caller's (device arrays):
 *   perm  int32[m], a permutation of 0..m-1 ((Pi_{m->m} x)_b = x_perm[b])
 *   phi   int8[m], +1 or -1 (the Rademacher signs of Phi)
 *   sel   int32[l], l distinct rows of the transform (Pi_{m->l})
 *   A, a_t, m, n, lda, X, x_t, ldx as for rpid_sketch; 1 <= l <= min(m, 1024)
 * Only l rows of the transform are kept, so the embedding is formed
 * explicitly (FP64 sincos, stored in A's type: BF16 rounds its entries) and
 * applied by the dense MFMA sketch.  Entries of perm outside [0, m) leave
 * their target columns of Gamma zero.
 */
int rpid_sketch_srtt(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n, int64_t lda,
                     const int32_t* perm, const int8_t* phi, const int32_t* sel, int64_t l, void* X,
                     rpid_dtype x_t, int64_t ldx);

/*
 * Sketch of a sparse A given in compressed sparse column form (the sparse
 * inputs of Sec. 5, e.g. eq. snn-def): X = Gamma A.
 *   colptr  int64[n + 1], rowidx int64[nnz], vals[nnz] of type v_t (F64 or
 *           F32), device; column j holds entries colptr[j] .. colptr[j+1]-1
 *           (pointers are clamped to [0, nnz]; row indices outside [0, m)
 *           are skipped)
 *   Gamma   l x m, ldg >= l, type v_t (dense embedding, e.g. Gaussian)
 *   X       l x n, ldx >= l, type v_t (output); 1 <= l <= 1024
 * Deterministic: each column's nonzeros are added in storage order.
 */
int rpid_sketch_csc(rpid_ctx ctx, const int64_t* colptr, const int64_t* rowidx, const void* vals,
                    rpid_dtype v_t, int64_t m, int64_t n, int64_t nnz, const void* Gamma, int64_t ldg,
                    int64_t l, void* X, int64_t ldx);

/*
 * The same CSC sketch with a sparse sign embedding (rows, signs, zeta, scale
 * as for rpid_sketch_sparse_sign); X is l x n of type v_t.  The embedding is
 * applied as the sparse operator of Sec. 2.2 (its cost in the table of
 * embedding costs is O(nnz zeta)): each nonzero a_ij adds +-a_ij into the zeta
 * rows of X(:, j) named by rows[i, :], nothing of size l x m is formed.
 * Deterministic: every row of X(:, j) receives its terms in the storage
 * order of column j, so the result has the bits of the CSC sketch with the
 * embedding written out densely (the zeta rows of one column of the
 * embedding must be distinct, as the definition has them; repeated rows are
 * not an error but then lose that property).  No workspace.
 */
int rpid_sketch_csc_sparse_sign(rpid_ctx ctx, const int64_t* colptr, const int64_t* rowidx,
                                const void* vals, rpid_dtype v_t, int64_t m, int64_t n, int64_t nnz,
                                const int32_t* rows, const int8_t* signs, int64_t zeta, int64_t l,
                                double scale, void* X, int64_t ldx);

/*
 * Dense columns of a CSC matrix: C(:, t) = A(:, J[t]) (m x k, ldc >= m, type
 * v_t), e.g. the skeleton C of a sparse A; J = NULL with k = n densifies all
 * of A.  Columns J[t] outside [0, n) come out as zeros.
 */
int rpid_csc_gather(rpid_ctx ctx, const int64_t* colptr, const int64_t* rowidx, const void* vals,
                    rpid_dtype v_t, int64_t m, int64_t n, int64_t nnz, int64_t k, const int64_t* J,
                    void* C, int64_t ldc);

/*
 * Rand-CPQR skeleton selection on the same sketch (the comparison pivoting
 * of Sec. 5; column-pivoted QR of eq. def_QRCP): k steps of Householder QR
 * with column pivoting on X.  Step t picks the remaining column with the
 * largest norm of its rows t..l-1 (ties to the smallest column), reflects it
 * to alpha e_t with alpha = -sign(x_t) ||x(t:l)||, and applies the reflector
 * to every remaining column; column norms are recomputed at every step.
 *   X, x_t (F64 or F32), l, n, ldx as for rpid_select_columns; 1 <= l <= 512,
 *   k <= min(l, n), n <= 32 x (compute units) (8192 on MI355X)
 *   J      int64[k]   pivots in pivot order (0-based columns of X)
 *   Rf     k x n, ldr >= k, type x_t: rows 0..k-1 of R in the original column
 *          order (Rf(t, J[t]) = alpha_t, Rf(t, J[s]) = 0 for s < t), so
 *          that X(:, J) = Q Rf(:, J) with orthonormal Q
 *   diagR  k values of type x_t: |Rf(t, J[t])|; may be NULL
 *   k_eff  host int64*, NULL to skip the synchronising status read
 * Returns 0, t + 1 when every remaining column is exactly zero in rows t..
 * (k_eff = t), RPID_ERR_NONFINITE for NaN/Inf in X, RPID_ERR_UNSUPPORTED for
 * sizes outside the limits above.
 */
int rpid_select_columns_cpqr(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n,
                             int64_t ldx, int64_t k, int64_t* J, void* Rf, int64_t ldr, void* diagR,
                             int64_t* k_eff);

/*
 * ID coefficients from the column-pivoted QR of the sketch: Z = R11^{-1} Rf
 * with R11 = Rf(:, J) (upper triangular in pivot order), so that Z(:, J) = I
 * and Z = X(:, J)^+ X (Sec. 4's estimate of C^+ A with all l rows).
 *   r_t    type of Rf (F64 or F32); k, n, J, Rf, ldr as returned by
 *          rpid_select_columns_cpqr
 *   Z      k x n FP64, ldz >= k (output)
 */
int rpid_id_coeffs_cpqr(rpid_ctx ctx, rpid_dtype r_t, int64_t k, int64_t n, const int64_t* J,
                        const void* Rf, int64_t ldr, double* Z, int64_t ldz);

/*
 * ID coefficients by least squares over all l rows of the sketch: Z = X_1^+ X
 * with X_1 = X(:, J) (l x k), Sec. 4's estimate of C^+ A taken literally for
 * l > k (rpid_id_coeffs uses the first k rows only; both agree for l = k).
 * Formed in FP64 by two Cholesky-QR passes of X_1 (X_1 = Q R) and
 * Z = R^{-1} (Q^T X), then Z(:, J) = I.
 *   X, x_t (F64 or F32), l, n, ldx, k, J as for rpid_id_coeffs (any pivots)
 *   Z      k x n FP64, ldz >= k (output)
 * Returns RPID_ERR_BREAKDOWN if a Cholesky factorisation meets a
 * non-positive pivot (X_1 numerically rank deficient); synchronises.
 */
int rpid_id_coeffs_ls(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n, int64_t ldx,
                      int64_t k, const int64_t* J, double* Z, int64_t ldz);

/*
 * S4 -- ID coefficients from the pivoted sketch (Sec. 4: C^+ A ~ X_1^+ X):
 * Z = X_1^{-1} X_k with X_k = X(0:k, :), X_1 = X_k(:, J), so that A ~ A(:, J) Z.
 * Computed from the LUPP factors: Z(:, J[t]) = e_t and, for j not in J,
 * Z(:, j) solves Lf(J, :)^T z = Lf(j, :)^T (unit upper triangular).
 * With refine_steps = 1, one step of iterative refinement in FP64 follows:
 * r = X_k(:, j) - X_1 z (X promoted to FP64), X_1 d = r solved through the
 * factors (Uf^T then Lf(J,:)^T), z += d.
 *   X, x_t, l, n, ldx, k, J, Lf, ldl, Uf, ldu as returned for rpid_select_columns
 *   Z      k x n FP64, ldz >= k (output)
 *   eta    host double*, NULL to skip: Theorem 1's a-posteriori factor
 *          sqrt(1 + ||Z_rest||_2^2), Z_rest = Z without the columns J
 *          (spectral norm by power iteration on Z_rest Z_rest^T to 1e-10
 *          relative change or 500 iterations)
 */
int rpid_id_coeffs(rpid_ctx ctx, const void* X, rpid_dtype x_t, int64_t l, int64_t n,
                   int64_t ldx, int64_t k, const int64_t* J, const void* Lf, int64_t ldl,
                   const void* Uf, int64_t ldu, double* Z, int64_t ldz, int refine_steps,
                   double* eta);

/*
 * S5-S7 -- CUR from the column skeleton (Alg. 2, step 4; eq. def_cur with
 * the stable construction eq. cur_stable):
 *   C = A(:, J) (pivot order); row-wise LUPP on C (k steps; ties to the
 *   smallest row; FP64 arithmetic if a_t = F64, else FP32) gives I;
 *   R = A(I, :); C = Q_C R_C, R^T = Q_R R_R (orthonormal Q by shifted
 *   Cholesky-QR in FP64); U = R_C^{-1} (Q_C^T A Q_R) R_R^{-T} in FP64, so
 *   that C U R = Q_C (Q_C^T A Q_R) Q_R^T.
 *   A      m x n, lda >= m, a_t in {F64, F32, BF16}
 *   J      int64[k] from rpid_select_columns (k <= 1024, k <= min(m, n))
 *   I      int64[k] (output)
 *   U      k x k FP64, ldu >= k (output)
 *   k_eff  host int64*, NULL to skip: rank reached by the row LUPP
 */
int rpid_cur(rpid_ctx ctx, const void* A, rpid_dtype a_t, int64_t m, int64_t n, int64_t lda,
             int64_t k, const int64_t* J, int64_t* I, double* U, int64_t ldu, int64_t* k_eff);

/*
 * S8 -- relative Frobenius error of the decomposition, by explicit
 * differences (the error measure of the experiments of Sec. 5):
 *   RPID_RESIDUAL_ID : ||A - A(:, J) Z||_F / ||A||_F   (uses J, Z)
 *   RPID_RESIDUAL_CUR: ||A - A(:, J) U A(I, :)||_F / ||A||_F (uses J, I, U)
 *   RPID_RESIDUAL_ROW_ID: ||A - Z^T A(I, :)||_F / ||A||_F (uses I, Z; Z is
 *     the k x m matrix that rpid_id_coeffs gives for the column sketch Yt of
 *     rpid_sketch_two_sided, i.e. the row ID A ~ A R^+ R estimated from the
 *     sketch as Y Y_1^+ after Alg. 3)
 * A is m x n of type a_t in {F64, F32, BF16}; Z is k x n (k x m for the row
 * ID) FP64 (ldz), U is k x k FP64 (ldu); unused arguments may be NULL.  The products run in FP64
 * for F64/F32 storage; for BF16 storage on BF16 MFMA with the FP64 factor
 * split into three BF16 terms and FP32 accumulation.  Sums of squares are
 * accumulated in FP64.  *rel_fro (host) receives the ratio; synchronises.
 */
int rpid_residual(rpid_ctx ctx, int which, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                  int64_t lda, int64_t k, const int64_t* J, const double* Z, int64_t ldz,
                  const int64_t* I, const double* U, int64_t ldu, double* rel_fro);

/*
 * The same residual without a host synchronisation: sums[0] = ||A - P Q||_F^2
 * and sums[1] = ||A||_F^2 (device FP64, caller-owned) are written on the
 * context's stream; the relative residual is sqrt(sums[0] / sums[1]).  For
 * overlapping it with other work on another stream.  Arguments as for
 * rpid_residual; -15 if sums is NULL.
 */
int rpid_residual_sums(rpid_ctx ctx, int which, const void* A, rpid_dtype a_t, int64_t m, int64_t n,
                       int64_t lda, int64_t k, const int64_t* J, const double* Z, int64_t ldz,
                       const int64_t* I, const double* U, int64_t ldu, double* sums);

/*
 * Learned rank (not in the paper).  Features of the pivot-magnitude profile
 * of a sketch's LUPP: f_t = max(log10(diagU[t] / diagU[0]), -20), t < L;
 * entries t >= k_eff (zero pivots) are -20.  diagU is type x_t (F32/F64),
 * feats is F32[L].
 */
int rpid_mlp_features(rpid_ctx ctx, const void* diagU, rpid_dtype x_t, int64_t L, int64_t k_eff,
                      float* feats);

/*
 * MLP 512 -> 128 -> 128 -> 1 (FP32, ReLU on the two hidden layers).
 * W is one flat device buffer of RPID_MLP_NPARAM floats:
 *   W1 (128 x 512, row-major), b1 (128), W2 (128 x 128), b2 (128), w3 (128), b3 (1).
 * forward : yhat[B] = net(feats[B x 512], row-major); act (nullable) receives
 *           the hidden activations needed by backward, B x 256 floats.
 * backward: dW = d(sum_b dy[b] * yhat[b]) / dW, accumulated over the batch
 *           (overwrites dW).
 * adam    : one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at step t >= 1.
 */
#define RPID_MLP_IN 512
#define RPID_MLP_H 128
#define RPID_MLP_NPARAM (128 * 512 + 128 + 128 * 128 + 128 + 128 + 1)
int rpid_mlp_forward(rpid_ctx ctx, const float* W, const float* feats, int64_t B, float* yhat,
                     float* act);
int rpid_mlp_backward(rpid_ctx ctx, const float* W, const float* feats, const float* act,
                      const float* dy, int64_t B, float* dW);
int rpid_mlp_adam(rpid_ctx ctx, float* W, const float* dW, float* m1, float* m2, float lr,
                  int64_t t);
/*
 * Training loss of the rank network: pinball (quantile) loss at level tau in
 * (0, 1) on targets log2 k*, r = target - yhat,
 *   loss = mean_b (tau max(r_b, 0) + (1 - tau) max(-r_b, 0)),
 * so that predicting a rank below k* (which costs a fallback) weighs tau /
 * (1 - tau) times more than predicting above it.  dy[B] (device) receives
 * d loss / d yhat (subgradient 0 at r = 0); *loss is one device float.
 */
int rpid_mlp_loss(rpid_ctx ctx, const float* yhat, const float* target, int64_t B, float tau,
                  float* dy, float* loss);

#ifdef __cplusplus
}
#endif

#endif /* RPID_H */
