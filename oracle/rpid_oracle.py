"""FP64 CPU oracle for randomized LUPP skeleton selection (ID and CUR).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module: only the tests, the smoke check and the CPU baseline leg of the
benchmark use it.  It shares no code with the HIP path.

Follows Dong & Martinsson, "Simpler is better: a comparative study of
randomized pivoting algorithms for CUR and interpolative decompositions":

* sketch            -- Alg. 2 (Randomized LUPP skeleton selection), step 2:
                       X = Gamma A with a Gaussian embedding Gamma (Sec. 2.2).
* sketch_power1     -- the row sketch with one plain power iteration,
                       eq. (def_power_iter) with q = 1: X = Omega A^T A.
* lupp_colwise      -- column-wise LU with partial pivoting of Sec. 2.4,
                       eq. (def_LUPP), Alg. 2 step 3.
* lupp_colwise_fma  -- the same steps in one fixed arithmetic (float64 or
                       float32, correctly rounded divisions, fused Schur
                       update), plain C in oracle/lupp_fma.c.
* id_coeffs         -- ID coefficients from the pivoted sketch, Sec. 4:
                       C^+ A is estimated by X_1^+ X (X_1 = X(:, J_s)).
* id_coeffs_ls      -- the same estimate by least squares over all l rows.
* eta               -- the a-posteriori factor of Theorem 1:
                       eta = || [-X_1^+ X_2 ; I] ||_2 = sqrt(1 + ||Z_rest||_2^2).
* lupp_rowwise      -- Alg. 2 step 4, row-wise LUPP on C = A(:, J_s).
* cur_u             -- U = C^+ A R^+ by the stable QR construction of the
                       Remark "Stable CUR", eq. (cur_stable).
* residuals         -- relative Frobenius errors of the ID A - C Z, the CUR
                       A - C U R, the optimal column ID A - C C^+ A (eq.
                       def_column_id), the row ID A - W R and the rangefinder
                       A - A X^+ X (Sec. 2.3).
* sketch_two_sided  -- Alg. 3 (streaming skeleton selection), step 2: the row
                       sketch X = Gamma A and the column sketch Y = A Omega^T.
* row_id_coeffs     -- the row ID estimated from the column sketch (after
                       Alg. 3): A R^+ is replaced by Y Y_1^+ (Y_1 = Y(I_s, :)).
* cur_sketch_u      -- the CUR core S^{-1}, S = A(I_s, J_s), that needs no
                       further pass over A (after Alg. 3).
* decompose_two_sided -- Alg. 3 end to end with the estimates above.
* cpqr_colwise      -- column-pivoted Householder QR of the sketch, eq.
                       (def_QRCP): the pivoting of Rand-CPQR (Sec. 5).
* id_coeffs_cpqr    -- Z = R_11^{-1} R_top from that QR (Z = X_1^+ X).
* sparse_sign_matrix, sketch_sparse_sign -- the sparse sign embedding of
                       Sec. 2.2 (zeta signed entries per column) and its sketch.
* dht_matrix, srtt_matrix, sketch_srtt -- the subsampled randomized
                       trigonometric transform of Sec. 2.2 with the discrete
                       Hartley transform.
* csc_dense, sketch_csc -- a matrix in compressed sparse column form (the
                       sparse inputs, eq. snn-def) and its sketch.

Everything is float64 numpy.  Library primitives used as single steps: matmul,
QR, triangular/linear solves, SVD (for spectral norms only).

Readings of the paper taken here (the paper is silent or garbled on them):
* argmax ties go to the smallest original index (eq. def_LUPP gives no rule);
* the first k pivots of a sketch with l >= k rows depend only on its first k
  rows (step t reads only row t of the updated sketch), so J_s(k) and Z(k)
  are computed from X(0:k, :);
* an exactly zero pivot stops the factorisation: status = t + 1 (1-based
  step of the zero pivot), k_eff = t (LAPACK getrf "info" convention);
* the Schur update of eq. (def_LUPP) is the standard one (the printed indices
  mix t and t + 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.linalg as sla

__all__ = [
    "sketch",
    "sketch_fp8",
    "e4m3_round",
    "fp8_scale_exp",
    "lupp_colwise",
    "lupp_colwise_fma",
    "lupp_rowwise",
    "id_coeffs",
    "id_coeffs_ls",
    "eta",
    "cur_u",
    "residuals",
    "rangefinder_error",
    "decompose",
    "sketch_power1",
    "sketch_two_sided",
    "row_id_coeffs",
    "cur_sketch_u",
    "decompose_two_sided",
    "cpqr_colwise",
    "id_coeffs_cpqr",
    "sparse_sign_matrix",
    "sketch_sparse_sign",
    "csc_dense",
    "sketch_csc",
    "dht_matrix",
    "srtt_matrix",
    "sketch_srtt",
    "NonFiniteInput",
]


class NonFiniteInput(ValueError):
    """Raised when a matrix handed to the pivoting step holds NaN or Inf."""


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Alg. 2, step 2: row sketch X = Gamma A
# --------------------------------------------------------------------------
def sketch(A, Omega):
    """X = Omega A (l x n) in float64 (Alg. 2, step 2)."""
    return _f64(Omega) @ _f64(A)


# --------------------------------------------------------------------------
# Row sketch with one plain power iteration, eq. (def_power_iter) with q = 1
# (the Rand-LUPP-1piter variant of Sec. 5): Omega is l x n here
# --------------------------------------------------------------------------
def sketch_power1(A, Omega):
    """X = Omega (A^T A) (l x n), formed as Y = A Omega^T (m x l) and then
    X = Y^T A, the order eq. (def_power_iter) implies for q = 1."""
    A = _f64(A)
    Y = A @ _f64(Omega).T
    return Y.T @ A


# --------------------------------------------------------------------------
# FP8 form of Alg. 2 step 2 (precision form, not in the paper): OCP E4M3
# operands with power-of-two scales, exact product of the quantised values
# --------------------------------------------------------------------------
E4M3_MAX = 448.0


def e4m3_values():
    """The 127 finite non-negative OCP E4M3 values in code order: exponent
    field e (bias 7) and 3-bit mantissa f; e = 0 is subnormal (f 2^-9);
    code 0x7F is NaN and there are no infinities."""
    vals = []
    for code in range(0x7F):
        e, f = code >> 3, code & 7
        vals.append(f * 2.0**-9 if e == 0 else (1.0 + f / 8.0) * 2.0 ** (e - 7))
    return np.array(vals)


def e4m3_round(x):
    """Round to the nearest E4M3 value, ties to the even code (|x| <= 448)."""
    x = _f64(x)
    table = e4m3_values()
    a = np.abs(x)
    hi = np.clip(np.searchsorted(table, a, side="left"), 0, table.size - 1)
    lo = np.clip(hi - 1, 0, table.size - 1)
    dlo, dhi = a - table[lo], table[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(a >= table[-1], table.size - 1, code)
    return np.sign(x) * table[code]


def fp8_scale_exp(mx):
    """Largest integer e with mx * 2^e <= 448 (0 for mx == 0)."""
    if not (mx > 0):
        return 0
    e = int(np.floor(np.log2(E4M3_MAX / mx)))
    while np.ldexp(mx, e + 1) <= E4M3_MAX:
        e += 1
    while np.ldexp(mx, e) > E4M3_MAX:
        e -= 1
    return e


def sketch_fp8(A, Omega):
    """X = (Om_q A_q) 2^-(eo + ea_j) with A_q(:, j) = e4m3(A(:, j) 2^ea_j) and
    Om_q = e4m3(Omega 2^eo), the exponents chosen per column of A and for
    all of Omega so that the largest modulus lands on or below 448."""
    A, Omega = _f64(A), _f64(Omega)
    ea = np.array([fp8_scale_exp(np.abs(A[:, j]).max()) for j in range(A.shape[1])])
    eo = fp8_scale_exp(np.abs(Omega).max())
    Aq = e4m3_round(A * np.ldexp(1.0, ea)[None, :])
    Oq = e4m3_round(Omega * np.ldexp(1.0, eo))
    return (Oq @ Aq) * np.ldexp(1.0, -(eo + ea))[None, :]


# --------------------------------------------------------------------------
# Sec. 2.4, eq. (def_LUPP): column-wise LU with partial pivoting
# --------------------------------------------------------------------------
def lupp_colwise(X, k, gaps=False):
    """k steps of column-wise LUPP on X (l x n), i.e. getrf of X^T.

    At step t (0-based) the pivot is the remaining column j with the largest
    |X^(t)(t, j)|; ties go to the smallest j.  The multipliers of step t are
    X^(t)(t, j) / X^(t)(t, p_t) (the entries of R^LU, all <= 1 in modulus),
    and the Schur complement update of eq. (def_LUPP) is applied to rows
    t+1..k-1 of the remaining columns.

    Returns a dict with
      J      int64[k_eff]  pivots in pivot order (0-based column indices of X)
      L      (n x k) float64, L[j, t] = multiplier of column j at step t
             (1 at the pivot's own step, 0 after it) = (R^LU)^T unpermuted
      U      (k x k) float64, U[t, :] = row t of the updated sketch at the
             pivot step, restricted to the first k rows (upper triangular
             as U[t, c] for c >= t holds X^(t)(c, p_t))
      diag   |U[t, t]|, the pivot magnitudes
      k_eff, status (0, or t+1 for an exactly zero pivot at step t)
      gap    (optional) relative gap between the largest and second-largest
             candidate magnitude at each step
    """
    X = _f64(X)
    l, n = X.shape
    if not (1 <= k <= min(l, n)):
        raise ValueError("need 1 <= k <= min(l, n)")
    if not np.isfinite(X[:k]).all():
        raise NonFiniteInput("non-finite entry in the sketch")
    # Work on the transpose: row j of S is column j of X (first k rows).
    S = X[:k, :].T.copy()
    remaining = np.ones(n, dtype=bool)
    J = []
    L = np.zeros((n, k))
    U = np.zeros((k, k))
    gap = []
    status = 0
    for t in range(k):
        cand = np.abs(S[:, t])
        cand[~remaining] = -1.0
        p = int(np.argmax(cand))  # first maximum: smallest index among ties
        piv = S[p, t]
        if gaps:
            c2 = cand.copy()
            c2[p] = -1.0
            second = c2.max()
            gap.append((abs(piv) - max(second, 0.0)) / abs(piv) if piv != 0 else 0.0)
        if piv == 0.0:
            status = t + 1
            break
        J.append(p)
        # U[c, t] = S[p, c] holds row c of X^(t) at the pivot column for c >= t.
        U[t, t:] = S[p, t:]
        remaining[p] = False
        L[p, t] = 1.0
        mult = S[remaining, t] / piv
        L[remaining, t] = mult
        S[np.ix_(remaining, np.arange(t + 1, k))] -= np.outer(mult, S[p, t + 1 : k])
    out = dict(
        J=np.array(J, dtype=np.int64),
        L=L,
        U=U,
        diag=np.abs(np.diag(U)),
        k_eff=len(J),
        status=status,
    )
    if gaps:
        out["gap"] = np.array(gap)
    return out


# --------------------------------------------------------------------------
# The same LUPP in one fixed arithmetic (oracle/lupp_fma.c): correctly
# rounded divisions and a fused (single-rounding) Schur update, in float64 or
# float32, so that a kernel doing the same operations can be compared bit for
# bit.  Compiled on first use with the host C compiler.
# --------------------------------------------------------------------------
_FMA_LIB = None
_HERE = os.path.dirname(os.path.abspath(__file__))
FMA_SRC = os.path.join(_HERE, "lupp_fma.c")
FMA_LIB = os.path.join(_HERE, "liblupp_fma.so")
FMA_CFLAGS = ["-O2", "-mfma", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared"]


def build_fma_lib(force=False):
    """Compile oracle/lupp_fma.c into oracle/liblupp_fma.so (contraction off:
    the only fused operations are the explicit fma calls)."""
    if force or not os.path.exists(FMA_LIB) or os.path.getmtime(FMA_LIB) < os.path.getmtime(FMA_SRC):
        cc = os.environ.get("CC", "gcc")
        tmp = FMA_LIB + ".tmp%d" % os.getpid()
        subprocess.run([cc, *FMA_CFLAGS, FMA_SRC, "-o", tmp, "-lm"], check=True, capture_output=True)
        os.replace(tmp, FMA_LIB)
    return FMA_LIB


def _fma_lib():
    global _FMA_LIB
    if _FMA_LIB is None:
        lib = ctypes.CDLL(build_fma_lib())
        P = ctypes.c_void_p
        for name in ("lupp_fma_f64", "lupp_fma_f32"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, P, P]
        _FMA_LIB = lib
    return _FMA_LIB


def lupp_colwise_fma(X, k, dtype=np.float64):
    """k steps of column-wise LUPP on X (l x n) as lupp_colwise, computed in
    `dtype` (float64 or float32) with m = S(i, t) / S(p, t) rounded once and
    the update S(i, c) = fma(-m, U(t, c), S(i, c)) rounded once.  X must be
    exactly representable in `dtype`.  Same return keys as lupp_colwise
    (L, U, diag in `dtype`)."""
    dtype = np.dtype(dtype)
    X = np.asarray(X)
    l, n = X.shape
    if not (1 <= k <= min(l, n)):
        raise ValueError("need 1 <= k <= min(l, n)")
    panel = np.ascontiguousarray(X[:k, :].T, dtype=dtype)
    if not np.array_equal(panel.astype(np.float64), np.asarray(X[:k, :].T, dtype=np.float64), equal_nan=True):
        raise ValueError("X is not exactly representable in %s" % dtype)
    J = np.zeros(k, dtype=np.int64)
    L = np.zeros((n, k), dtype=dtype)
    U = np.zeros((k, k), dtype=dtype)
    diag = np.zeros(k, dtype=dtype)
    fn = _fma_lib().lupp_fma_f64 if dtype == np.float64 else _fma_lib().lupp_fma_f32
    st = fn(n, k, panel.ctypes.data, J.ctypes.data, L.ctypes.data, U.ctypes.data, diag.ctypes.data)
    if st == -1:
        raise NonFiniteInput("non-finite entry in the sketch")
    if st < -1:
        raise MemoryError("lupp_fma")
    k_eff = k if st == 0 else st - 1
    return dict(J=J[:k_eff], L=L, U=U, diag=diag[:k_eff], k_eff=k_eff, status=st)


def lupp_rowwise(C, k, gaps=False):
    """k steps of row-wise LUPP on C (m x k'), i.e. column-wise LUPP on C^T
    (Alg. 2, step 4).  Pivots are row indices of C."""
    return lupp_colwise(_f64(C).T, k, gaps=gaps)


# --------------------------------------------------------------------------
# Sec. 4: ID coefficients from the pivoted sketch, and Theorem 1's eta
# --------------------------------------------------------------------------
def id_coeffs(X, J, k=None):
    """Z (k x n) with A ~ A(:, J) Z, estimated from the sketch: Z = X_1^{-1} X_k
    where X_k = X(0:k, :) and X_1 = X_k(:, J) (Sec. 4).  Z(:, J) = I exactly."""
    X = _f64(X)
    J = np.asarray(J, dtype=np.int64)
    if k is None:
        k = J.shape[0]
    J = J[:k]
    Xk = X[:k, :]
    Z = np.linalg.solve(Xk[:, J], Xk)
    Z[:, J] = np.eye(k)
    return Z


def id_coeffs_ls(X, J, k=None):
    """Z = X(:, J)^+ X by least squares over all l rows of the sketch (Sec.
    4's X_1^+ X for l > k); Z(:, J) = I."""
    X = _f64(X)
    J = np.asarray(J, dtype=np.int64)
    if k is None:
        k = J.shape[0]
    J = J[:k]
    Z = np.linalg.lstsq(X[:, J], X, rcond=None)[0]
    Z[:, J] = np.eye(k)
    return Z


def rest_of(n, J):
    mask = np.ones(n, dtype=bool)
    mask[np.asarray(J, dtype=np.int64)] = False
    return np.nonzero(mask)[0]


def eta(Z, J):
    """Theorem 1: eta = ||[-X_1^+ X_2; I]||_2 = sqrt(1 + ||Z_rest||_2^2)."""
    Z = _f64(Z)
    rest = rest_of(Z.shape[1], J)
    if rest.size == 0:
        return 1.0
    s = np.linalg.norm(Z[:, rest], 2)
    return float(np.sqrt(1.0 + s * s))


# --------------------------------------------------------------------------
# Remark "Stable CUR": U = C^+ A R^+ through unpivoted QR of C and R^T
# --------------------------------------------------------------------------
def cur_u(A, J, I):
    """U (k x k) such that C U R = Q_C (Q_C^T A Q_R) Q_R^T (eq. cur_stable)."""
    A = _f64(A)
    C = A[:, J]
    R = A[I, :]
    qc, rc = np.linalg.qr(C)
    qr_, rr = np.linalg.qr(R.T)
    M = qc.T @ A @ qr_
    # U = R_C^{-1} M R_R^{-T}
    U = sla.solve_triangular(rc, M, lower=False)
    U = sla.solve_triangular(rr, U.T, lower=False).T
    return U


# --------------------------------------------------------------------------
# Error metrics
# --------------------------------------------------------------------------
def _fro(a):
    return float(np.sqrt(np.sum(np.square(a))))


def rangefinder_error(A, X, k, ord="fro"):
    """||A - A X_k^+ X_k|| / ||A|| (Sec. 2.3), X_k = X(0:k, :)."""
    A = _f64(A)
    q, _ = np.linalg.qr(_f64(X)[:k, :].T)
    E = A - (A @ q) @ q.T
    if ord == "fro":
        return _fro(E) / _fro(A)
    return float(np.linalg.norm(E, 2) / np.linalg.norm(A, 2))


def residuals(A, J, Z=None, I=None, U=None, ord="fro", only=None, W=None):
    """Relative errors; explicit differences (never an expanded form).

    id    ||A - A(:,J) Z|| / ||A||          (Z from the sketch, Sec. 4)
    idopt ||A - C C^+ A|| / ||A||           (eq. def_column_id)
    cur   ||A - C U R|| / ||A||             (eq. def_cur)
    rowopt||A - A R^+ R|| / ||A||           (eq. def_row_id)
    rowid ||A - W A(I,:)|| / ||A||          (W from the column sketch)
    ``only`` (optional) restricts the work to the listed keys; J may be None
    when only row quantities are asked for.
    """
    A = _f64(A)
    nrm = (lambda e: _fro(e)) if ord == "fro" else (lambda e: float(np.linalg.norm(e, 2)))
    na = nrm(A)
    C = A[:, J] if J is not None else None
    want = (lambda key: only is None or key in only)
    out = {}
    if C is not None and want("idopt"):
        qc, _ = np.linalg.qr(C)
        out["idopt"] = nrm(A - qc @ (qc.T @ A)) / na
    if Z is not None and want("id"):
        out["id"] = nrm(A - C @ _f64(Z)) / na
    if I is not None:
        R = A[I, :]
        if want("rowopt"):
            qr_, _ = np.linalg.qr(R.T)
            out["rowopt"] = nrm(A - (A @ qr_) @ qr_.T) / na
        if U is not None and want("cur"):
            out["cur"] = nrm(A - (C @ _f64(U)) @ R) / na
        if W is not None and want("rowid"):
            out["rowid"] = nrm(A - _f64(W) @ R) / na
    return out


def optimal_error(s, k):
    """||A - A_k||_F / ||A||_F from the singular values s (Eckart-Young)."""
    s = np.asarray(s, dtype=np.float64)
    return float(np.sqrt(np.sum(s[k:] ** 2) / np.sum(s**2)))


# --------------------------------------------------------------------------
# The whole path of Alg. 2 with the sketch-based ID and stable CUR
# --------------------------------------------------------------------------
def decompose(A, Omega, k, gaps=False, want_cur=True, lupp="numpy", X=None):
    """Alg. 2 end to end: X = Omega A; LUPP on X -> J; Z; C = A(:, J);
    LUPP on C -> I; U.  Returns a dict with every intermediate.
    lupp="fma" takes both LUPPs from lupp_colwise_fma in float64 (no gaps);
    X (optional) replaces the sketch (e.g. the FP8 form's)."""
    A = _f64(A)
    X = sketch(A, Omega) if X is None else _f64(X)
    if lupp == "fma":
        if gaps:
            raise ValueError("gaps need the numpy LUPP")
        lupp_colwise_ = lambda X_, k_, gaps=False: lupp_colwise_fma(X_, k_, np.float64)  # noqa: E731
    else:
        lupp_colwise_ = lupp_colwise
    col = lupp_colwise_(X, k, gaps=gaps)
    out = dict(X=X, J=col["J"], L=col["L"], Ufac=col["U"], diag=col["diag"],
               k_eff=col["k_eff"], status=col["status"])
    if gaps:
        out["gap_J"] = col["gap"]
    if col["status"] != 0:
        return out
    J = col["J"]
    Z = id_coeffs(X, J, k)
    out["Z"] = Z
    out["eta"] = eta(Z, J)
    if want_cur:
        C = A[:, J]
        row = lupp_colwise_(C.T, k, gaps=gaps)
        out["I"] = row["J"]
        out["status_I"] = row["status"]
        if gaps:
            out["gap_I"] = row["gap"]
        if row["status"] == 0:
            out["U"] = cur_u(A, J, row["J"])
    return out


# --------------------------------------------------------------------------
# Alg. 3: streaming (two-sided, single-pass) skeleton selection, and the
# estimates of the ID and CUR that avoid a further pass over A
# --------------------------------------------------------------------------
def sketch_two_sided(A, Gamma, Omega):
    """Alg. 3, step 2 with independent embeddings Gamma (l x m) and Omega
    (l x n): X = Gamma A (l x n) and Y = A Omega^T (m x l)."""
    A = _f64(A)
    return _f64(Gamma) @ A, A @ _f64(Omega).T


def row_id_coeffs(Y, I, k=None):
    """W (m x k) with A ~ W A(I, :), estimated from the column sketch: A R^+
    is replaced by Y Y_1^+ with Y_1 = Y(I, :).  With k < l the first k
    columns are used, Y_k = Y(:, 0:k) and W = Y_k Y_k(I, :)^{-1} (the row
    analogue of Z in Sec. 4); W(I, :) = I exactly."""
    Y = _f64(Y)
    I = np.asarray(I, dtype=np.int64)
    if k is None:
        k = I.shape[0]
    I = I[:k]
    Yk = Y[:, :k]
    # W Y_1 = Y_k  <=>  Y_1^T W^T = Y_k^T
    W = np.linalg.solve(Yk[I, :].T, Yk.T).T
    W[I, :] = np.eye(k)
    return W


def cur_sketch_u(A, J, I):
    """U = S^{-1} with S = A(I, J), the core of the CUR C S^{-1} R."""
    A = _f64(A)
    S = A[np.ix_(np.asarray(I, dtype=np.int64), np.asarray(J, dtype=np.int64))]
    return np.linalg.solve(S, np.eye(S.shape[0]))


def decompose_two_sided(A, Gamma, Omega, k, gaps=False):
    """Alg. 3: both sketches, column LUPP on X -> J, row LUPP on Y -> I; then
    Z from X (Sec. 4), W from Y, the cheap core S^{-1} and the stable core
    C^+ A R^+ for comparison."""
    A = _f64(A)
    X, Y = sketch_two_sided(A, Gamma, Omega)
    col = lupp_colwise(X, k, gaps=gaps)
    row = lupp_rowwise(Y, k, gaps=gaps)
    out = dict(X=X, Y=Y, J=col["J"], I=row["J"], status_J=col["status"], status_I=row["status"])
    if gaps:
        out["gap_J"], out["gap_I"] = col["gap"], row["gap"]
    if col["status"] != 0 or row["status"] != 0:
        return out
    out["Z"] = id_coeffs(X, col["J"], k)
    out["W"] = row_id_coeffs(Y, row["J"], k)
    out["U_sketch"] = cur_sketch_u(A, col["J"], row["J"])
    out["U"] = cur_u(A, col["J"], row["J"])
    return out


# --------------------------------------------------------------------------
# Rand-CPQR (Sec. 5): column-pivoted QR, eq. (def_QRCP), on the same sketch
# --------------------------------------------------------------------------
def cpqr_colwise(X, k, gaps=False):
    """k steps of Householder QR with column pivoting on X (l x n).

    At step t the pivot is the remaining column whose rows t..l-1 (of the
    matrix updated by the earlier reflectors) have the largest Euclidean norm,
    ties to the smallest column; the norms are computed afresh at every step.
    The reflector of the pivot column w = X^(t)(t:, p) maps it to alpha e_0
    with alpha = -sign(w_0) ||w|| (sign(0) = +1): v = w - alpha e_0,
    beta = 1 / (alpha (alpha - w_0)), and every remaining column x gets
    x(t:) -= beta (v^T x(t:)) v.  Row t of R is row t after that update.

    Returns a dict with J (pivots in order), R (k x n, original column order;
    R[t, J[t]] = alpha_t, zero at the earlier pivots), diag = |alpha_t|,
    k_eff, status (t + 1 when every remaining column is zero in rows t..)
    and, with gaps=True, the relative gap between the two largest norms at
    each step.
    """
    S = _f64(X).copy()
    if not np.all(np.isfinite(S)):
        raise NonFiniteInput("non-finite entry in the sketch")
    l, n = S.shape
    remaining = np.ones(n, dtype=bool)
    R = np.zeros((k, n))
    J, gap = [], []
    status = 0
    for t in range(k):
        norms = np.sqrt(np.sum(S[t:, :] ** 2, axis=0))
        cand = np.where(remaining, norms, -1.0)
        p = int(cand.argmax())  # the first maximum
        if not cand[p] > 0.0:
            status = t + 1
            break
        if gaps:
            others = np.delete(cand, p)
            second = others.max() if others.size else -1.0
            gap.append((cand[p] - max(second, 0.0)) / cand[p])
        w = S[t:, p].copy()
        alpha = -np.linalg.norm(w) if w[0] >= 0.0 else np.linalg.norm(w)
        v = w.copy()
        v[0] -= alpha
        beta = 1.0 / (alpha * (alpha - w[0]))
        cols = remaining.copy()
        cols[p] = False
        d = v @ S[t:, cols]
        S[t:, cols] -= beta * np.outer(v, d)
        R[t, cols] = S[t, cols]
        R[t, p] = alpha
        S[t:, p] = 0.0
        remaining[p] = False
        J.append(p)
    out = dict(J=np.array(J, dtype=np.int64), R=R, diag=np.abs(np.array([R[t, J[t]] for t in range(len(J))])),
               k_eff=len(J), status=status)
    if gaps:
        out["gap"] = np.array(gap)
    return out


def id_coeffs_cpqr(R, J):
    """Z = R_11^{-1} R with R_11 = R(:, J): the ID coefficients of the
    column-pivoted QR (equal to X(:, J)^+ X for the sketch X)."""
    R = _f64(R)
    J = np.asarray(J, dtype=np.int64)
    k = J.shape[0]
    Z = sla.solve_triangular(R[:k, J], R[:k, :], lower=False)
    Z[:, J] = np.eye(k)
    return Z


# --------------------------------------------------------------------------
# Sec. 2.2: sparse sign embeddings; sparse A in compressed sparse column form
# --------------------------------------------------------------------------
def sparse_sign_matrix(rows, signs, l):
    """The l x m sparse sign embedding (unscaled): column i holds signs[i, s]
    at row rows[i, s] for s < zeta and zeros elsewhere."""
    rows = np.asarray(rows)
    signs = np.asarray(signs)
    m, zeta = rows.shape
    G = np.zeros((l, m))
    for i in range(m):
        for s_ in range(zeta):
            G[rows[i, s_], i] = float(signs[i, s_])
    return G


def sketch_sparse_sign(A, rows, signs, l, scale):
    """X = scale * S A with S = sparse_sign_matrix(rows, signs, l)."""
    return float(scale) * (sparse_sign_matrix(rows, signs, l) @ _f64(A))


def csc_dense(colptr, rowidx, vals, m, n):
    """The dense m x n matrix whose column j holds vals[p] at row rowidx[p]
    for colptr[j] <= p < colptr[j + 1]."""
    A = np.zeros((m, n))
    for j in range(n):
        for p in range(int(colptr[j]), int(colptr[j + 1])):
            A[int(rowidx[p]), j] = float(vals[p])
    return A


def sketch_csc(colptr, rowidx, vals, m, n, Gamma):
    """X = Gamma A for A given in compressed sparse column form."""
    return _f64(Gamma) @ csc_dense(colptr, rowidx, vals, m, n)


def dht_matrix(m):
    """The m x m unitary discrete Hartley transform, T(a, b) = cas(2 pi a b /
    m) / sqrt(m) with cas = cos + sin (a, b = 0..m-1)."""
    ab = np.outer(np.arange(m), np.arange(m)) % m
    ang = 2.0 * np.pi * ab / m
    return (np.cos(ang) + np.sin(ang)) / np.sqrt(m)


def srtt_matrix(perm, phi, sel, m, l):
    """Gamma = sqrt(m / l) Pi_{m->l} T Phi Pi_{m->m} (Sec. 2.2): (Pi_{m->m} x)_b
    = x_{perm[b]}, Phi = diag(phi), T the DHT, (Pi_{m->l} z)_r = z_{sel[r]}."""
    P = np.zeros((m, m))
    P[np.arange(m), np.asarray(perm)] = 1.0
    S = np.zeros((l, m))
    S[np.arange(l), np.asarray(sel)] = 1.0
    return np.sqrt(m / l) * (S @ dht_matrix(m) @ np.diag(np.asarray(phi, dtype=np.float64)) @ P)


def sketch_srtt(A, perm, phi, sel, l):
    """X = Gamma A with the SRTT embedding above."""
    A = _f64(A)
    return srtt_matrix(perm, phi, sel, A.shape[0], l) @ A
