/*
 * TEST INFRASTRUCTURE ONLY -- part of the CPU oracle; nothing in the product
 * path may link or call it.  Shares no code with the HIP library.
 *
 * Column-wise LU with partial pivoting of a sketch, k steps (eq. def_LUPP of
 * Dong & Martinsson, Alg. 2 step 3), written as a plain triple loop in one
 * fixed arithmetic so that its every value can be compared bit for bit:
 *
 *   panel S = X(0:k, :)^T, n x k, row i = candidate (column i of X);
 *   step t: p = argmax over remaining i of |S[i][t]| (ties: smallest i);
 *           stop with status t + 1 if S[p][t] == 0;
 *           U[t][c] = S[p][c] for c >= t;
 *           m_i = S[i][t] / S[p][t]     (one correctly rounded division)
 *           S[i][c] = fma(-m_i, U[t][c], S[i][c])  for c > t, remaining i
 *                                        (one rounding per update)
 *
 * The single rounding of the Schur update (a fused multiply-add) is the
 * reading of the update's arithmetic that this variant fixes; the numpy
 * oracle keeps the unfused form (a product rounded, then a difference
 * rounded).  Both are the same algorithm; they can differ in the last bit of
 * an entry, and hence in a pivot only where two candidates tie to within
 * rounding.
 *
 * Layout: S (input) is n x k row-major (S[i * k + c]); L (output) is n x k
 * row-major with L[i][t] = m_i for rows remaining at step t, 1 at the pivot
 * row, 0 for rows pivoted earlier; U is k x k row-major, zero below the
 * diagonal; J[t] = pivot row of step t; diag[t] = |U[t][t]|.
 * Returns 0, t + 1 for an exactly zero pivot at step t (only t pivots are
 * defined), or -1 if S holds a NaN or an infinity.
 *
 * The rows of one step are independent, so they are updated in parallel
 * (OpenMP); every value is the same for any thread count.
 *
 * Build: cc -O2 -mfma -fopenmp -ffp-contract=off -fPIC -shared lupp_fma.c
 *        -o liblupp_fma.so -lm
 * (contraction off: the only fused operations are the explicit fma calls,
 * which -mfma turns into the hardware instruction, itself a single rounding).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DEFINE_LUPP(NAME, T, FMA, FABS, ISFINITE)                                         \
  int NAME(int64_t n, int64_t k, const T* S_in, int64_t* J, T* L, T* U, T* diag) {        \
    T* S = (T*)malloc(sizeof(T) * (size_t)n * (size_t)k);                                 \
    unsigned char* done = (unsigned char*)calloc((size_t)n, 1);                           \
    if (!S || !done) {                                                                    \
      free(S);                                                                            \
      free(done);                                                                         \
      return -2;                                                                          \
    }                                                                                     \
    memcpy(S, S_in, sizeof(T) * (size_t)n * (size_t)k);                                   \
    for (int64_t i = 0; i < n * k; ++i) {                                                 \
      if (!ISFINITE(S[i])) {                                                              \
        free(S);                                                                          \
        free(done);                                                                       \
        return -1;                                                                        \
      }                                                                                   \
    }                                                                                     \
    memset(L, 0, sizeof(T) * (size_t)n * (size_t)k);                                      \
    memset(U, 0, sizeof(T) * (size_t)k * (size_t)k);                                      \
    int status = 0;                                                                       \
    for (int64_t t = 0; t < k; ++t) {                                                     \
      int64_t p = -1;                                                                     \
      T best = (T)-1;                                                                     \
      for (int64_t i = 0; i < n; ++i) {                                                   \
        if (done[i]) continue;                                                            \
        T a = FABS(S[i * k + t]);                                                         \
        if (a > best) { /* strictly larger: ties keep the smaller i */                    \
          best = a;                                                                       \
          p = i;                                                                          \
        }                                                                                 \
      }                                                                                   \
      if (p < 0 || best == (T)0) {                                                        \
        status = (int)(t + 1);                                                            \
        break;                                                                            \
      }                                                                                   \
      const T piv = S[p * k + t];                                                         \
      J[t] = p;                                                                           \
      diag[t] = FABS(piv);                                                                \
      for (int64_t c = t; c < k; ++c) U[t * k + c] = S[p * k + c];                        \
      done[p] = 1;                                                                        \
      L[p * k + t] = (T)1;                                                                \
      _Pragma("omp parallel for schedule(static)")                                        \
      for (int64_t i = 0; i < n; ++i) {                                                   \
        if (done[i]) continue;                                                            \
        const T m = S[i * k + t] / piv;                                                   \
        L[i * k + t] = m;                                                                 \
        for (int64_t c = t + 1; c < k; ++c) S[i * k + c] = FMA(-m, U[t * k + c], S[i * k + c]); \
      }                                                                                   \
    }                                                                                     \
    free(S);                                                                              \
    free(done);                                                                           \
    return status;                                                                        \
  }

DEFINE_LUPP(lupp_fma_f64, double, fma, fabs, isfinite)
DEFINE_LUPP(lupp_fma_f32, float, fmaf, fabsf, isfinite)
