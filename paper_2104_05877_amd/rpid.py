"""Thin ctypes binding of librpid (include/rpid.h): argument marshalling only.

Every function carries the name of the C entry point it calls.  Matrices are
torch tensors on the GPU in column-major layout: an m x n matrix is a tensor
``t`` of shape (m, n) with ``t.stride() == (1, ld)``, ``ld >= m`` (e.g. the
transpose of a contiguous (n, m) tensor).  Index vectors are int64 tensors.
All calls enqueue on the stream given to :class:`Context` (by default torch's
current stream).  Outputs are allocated by torch on its current stream: with a
context on another stream, keep them alive until that stream has been
synchronised (or mark them with ``Tensor.record_stream``), or torch may hand
their memory out again while the context's kernels still write it.  There is
no fallback: if the HIP library is missing or the GPU is absent, the calls
raise.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpid.so")

F64, F32, BF16, FP8_E4M3 = 0, 1, 2, 3
RESIDUAL_ID, RESIDUAL_CUR, RESIDUAL_ROW_ID = 0, 1, 2
MLP_IN, MLP_H = 512, 128
MLP_NPARAM = 128 * 512 + 128 + 128 * 128 + 128 + 128 + 1

ERR = {
    -100: "NONFINITE",
    -101: "HIP",
    -102: "NOMEM",
    -103: "UNSUPPORTED",
    -104: "LAUNCH",
    -105: "TIMEOUT",
    -106: "BREAKDOWN",
    -107: "SCRATCH",
}

_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int64
_i = ctypes.c_int

_SIGS = {
    "rpid_create": (_i, [ctypes.POINTER(_P), _i, _P]),
    "rpid_destroy": (_i, [_P]),
    "rpid_set_stream": (_i, [_P, _P]),
    "rpid_status_string": (ctypes.c_char_p, [_i]),
    "rpid_version": (_i, []),
    "rpid_sketch": (_i, [_P, _P, _i, _I, _I, _I, _P, _i, _I, _I, _P, _i, _I]),
    "rpid_sketch_noalloc": (_i, [_P, _P, _i, _I, _I, _I, _P, _i, _I, _I, _P, _i, _I]),
    "rpid_sketch_power1": (_i, [_P, _P, _i, _I, _I, _I, _P, _i, _I, _I, _P, _i, _I]),
    "rpid_sketch_two_sided": (_i, [_P, _P, _i, _I, _I, _I, _P, _I, _P, _I, _I, _P, _I, _P, _I, _i]),
    "rpid_cur_sketch": (_i, [_P, _P, _i, _I, _I, _I, _I, _P, _P, _P, _I]),
    "rpid_select_columns_cpqr": (_i, [_P, _P, _i, _I, _I, _I, _I, _P, _P, _I, _P, _P]),
    "rpid_sketch_sparse_sign": (_i, [_P, _P, _i, _I, _I, _I, _P, _P, _I, _I, ctypes.c_double, _P, _i, _I]),
    "rpid_sketch_csc": (_i, [_P, _P, _P, _P, _i, _I, _I, _I, _P, _I, _I, _P, _I]),
    "rpid_sketch_srtt": (_i, [_P, _P, _i, _I, _I, _I, _P, _P, _P, _I, _P, _i, _I]),
    "rpid_sketch_csc_sparse_sign": (_i, [_P, _P, _P, _P, _i, _I, _I, _I, _P, _P, _I, _I, ctypes.c_double,
                                         _P, _I]),
    "rpid_csc_gather": (_i, [_P, _P, _P, _P, _i, _I, _I, _I, _I, _P, _P, _I]),
    "rpid_id_coeffs_cpqr": (_i, [_P, _i, _I, _I, _P, _P, _I, _P, _I]),
    "rpid_id_coeffs_ls": (_i, [_P, _P, _i, _I, _I, _I, _I, _P, _P, _I]),
    "rpid_sketch_fp8": (_i, [_P, _P, _I, _I, _I, _P, _I, _I, _P, _I]),
    "rpid_select_columns": (_i, [_P, _P, _i, _I, _I, _I, _I, _P, _P, _I, _P, _I, _P, ctypes.POINTER(_I)]),
    "rpid_select_columns_async": (_i, [_P, _P, _i, _I, _I, _I, _I, _P, _P, _I, _P, _I, _P, _P]),
    "rpid_id_coeffs": (
        _i,
        [_P, _P, _i, _I, _I, _I, _I, _P, _P, _I, _P, _I, _P, _I, _i, ctypes.POINTER(ctypes.c_double)],
    ),
    "rpid_cur": (_i, [_P, _P, _i, _I, _I, _I, _I, _P, _P, _P, _I, ctypes.POINTER(_I)]),
    "rpid_residual_sums": (_i, [_P, _i, _P, _i, _I, _I, _I, _I, _P, _P, _I, _P, _P, _I, _P]),
    "rpid_residual": (
        _i,
        [_P, _i, _P, _i, _I, _I, _I, _I, _P, _P, _I, _P, _P, _I, ctypes.POINTER(ctypes.c_double)],
    ),
    "rpid_mlp_features": (_i, [_P, _P, _i, _I, _I, _P]),
    "rpid_mlp_forward": (_i, [_P, _P, _P, _I, _P, _P]),
    "rpid_mlp_backward": (_i, [_P, _P, _P, _P, _P, _I, _P]),
    "rpid_mlp_adam": (_i, [_P, _P, _P, _P, _P, ctypes.c_float, _I]),
    "rpid_mlp_loss": (_i, [_P, _P, _P, _I, ctypes.c_float, _P, _P]),
}


class RpidError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        name = ERR.get(status, f"argument {-status} invalid" if status < 0 else "zero pivot")
        super().__init__(f"{fn} failed with status {status} ({name})")


def lib():
    """Load librpid.so (built in-tree by paper_2104_05877_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library not built: {LIB_PATH} is missing "
                "(run python -m paper_2104_05877_amd.build)"
            )
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def symbols():
    """Names of the entry points the binding expects the library to export."""
    return list(_SIGS)


def _check(fn, status, allow_positive=False):
    if status < 0 or (status > 0 and not allow_positive):
        raise RpidError(fn, status)
    return status


def dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported dtype {t.dtype}")


def colmajor(t: torch.Tensor):
    """(pointer, rows, cols, ld) of a column-major GPU matrix."""
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    rows, cols = t.shape
    if t.stride(0) != 1 and rows > 1:
        raise ValueError("matrix must be column-major (stride(0) == 1)")
    ld = t.stride(1) if cols > 1 else max(rows, 1)
    if ld < rows:
        raise ValueError("leading dimension smaller than the row count")
    return t.data_ptr(), rows, cols, ld


def empty_colmajor(rows, cols, dtype, device):
    return torch.empty((cols, rows), dtype=dtype, device=device).T


class Context:
    """An rpid context bound to a device and a HIP stream (torch's current
    stream by default)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = _P()
        _check("rpid_create", L.rpid_create(ctypes.byref(h), device, _P(stream.cuda_stream)))
        self.handle = h

    def close(self):
        worker = self.__dict__.pop("_side_worker", None)
        if worker is not None:
            worker.stop()
        if self.handle:
            lib().rpid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def rpid_sketch(ctx: Context, A: torch.Tensor, Omega: torch.Tensor, out_dtype=None) -> torch.Tensor:
    """X = Omega A (Alg. 2, step 2).  BF16 inputs give an FP32 X."""
    pa, m, n, lda = colmajor(A)
    po, l, m2, ldo = colmajor(Omega)
    if m2 != m:
        raise ValueError("Omega must have m columns")
    if out_dtype is None:
        out_dtype = torch.float32 if A.dtype == torch.bfloat16 else A.dtype
    X = empty_colmajor(l, n, out_dtype, A.device)
    px, _, _, ldx = colmajor(X)
    s = lib().rpid_sketch(ctx.handle, pa, dtype_code(A), m, n, lda, po, dtype_code(Omega), l, ldo, px,
                          dtype_code(X), ldx)
    _check("rpid_sketch", s)
    return X


def rpid_sketch_noalloc(ctx: Context, A: torch.Tensor, Omega: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """X = Omega A into the caller's X (l x n, column-major; FP32 for BF16
    inputs) with the library's fixed device scratch: the call allocates
    nothing."""
    pa, m, n, lda = colmajor(A)
    po, l, m2, ldo = colmajor(Omega)
    px, lx, nx, ldx = colmajor(X)
    if m2 != m or lx != l or nx != n:
        raise ValueError("shapes of A (m x n), Omega (l x m) and X (l x n) disagree")
    s = lib().rpid_sketch_noalloc(ctx.handle, pa, dtype_code(A), m, n, lda, po, dtype_code(Omega), l,
                                  ldo, px, dtype_code(X), ldx)
    _check("rpid_sketch_noalloc", s)
    return X


def rpid_sketch_power1(ctx: Context, A: torch.Tensor, Omega: torch.Tensor) -> torch.Tensor:
    """X = Omega A^T A (one plain power iteration); Omega is l x n.  BF16
    inputs give an FP32 X."""
    pa, m, n, lda = colmajor(A)
    po, l, n2, ldo = colmajor(Omega)
    if n2 != n:
        raise ValueError("Omega must have n columns")
    out_dtype = torch.float32 if A.dtype == torch.bfloat16 else A.dtype
    X = empty_colmajor(l, n, out_dtype, A.device)
    px, _, _, ldx = colmajor(X)
    s = lib().rpid_sketch_power1(ctx.handle, pa, dtype_code(A), m, n, lda, po, dtype_code(Omega), l, ldo,
                                 px, dtype_code(X), ldx)
    _check("rpid_sketch_power1", s)
    return X


def rpid_sketch_two_sided(ctx: Context, A: torch.Tensor, Gamma: torch.Tensor, Omega: torch.Tensor):
    """Alg. 3, step 2: X = Gamma A (l x n) and Yt = Omega A^T (l x m, the
    column sketch Y = A Omega^T transposed).  Gamma is l x m, Omega l x n.
    BF16 inputs give FP32 sketches."""
    pa, m, n, lda = colmajor(A)
    pg, l, m2, ldg = colmajor(Gamma)
    po, l2, n2, ldo = colmajor(Omega)
    if m2 != m or n2 != n or l2 != l:
        raise ValueError("Gamma must be l x m and Omega l x n")
    if Gamma.dtype != A.dtype or Omega.dtype != A.dtype:
        raise ValueError("Gamma and Omega must have A's dtype")
    out_dtype = torch.float64 if A.dtype == torch.float64 else torch.float32
    X = empty_colmajor(l, n, out_dtype, A.device)
    Yt = empty_colmajor(l, m, out_dtype, A.device)
    px, _, _, ldx = colmajor(X)
    py, _, _, ldy = colmajor(Yt)
    s = lib().rpid_sketch_two_sided(ctx.handle, pa, dtype_code(A), m, n, lda, pg, ldg, po, ldo, l, px, ldx,
                                    py, ldy, dtype_code(X))
    _check("rpid_sketch_two_sided", s)
    return X, Yt


def rpid_cur_sketch(ctx: Context, A: torch.Tensor, k: int, J: torch.Tensor, I: torch.Tensor):
    """U = A(I, J)^{-1} (k x k FP64), the sketch-only CUR core.  Returns
    (U, status); status > 0 reports an exactly zero pivot of A(I, J)."""
    pa, m, n, lda = colmajor(A)
    U = empty_colmajor(k, k, torch.float64, A.device)
    s = lib().rpid_cur_sketch(ctx.handle, pa, dtype_code(A), m, n, lda, k, J.data_ptr(), I.data_ptr(),
                              U.data_ptr(), U.stride(1))
    _check("rpid_cur_sketch", s, allow_positive=True)
    return U, s


def rpid_sketch_fp8(ctx: Context, A: torch.Tensor, Omega: torch.Tensor) -> torch.Tensor:
    """FP8 (E4M3, power-of-two scaled) sketch of FP32 A; FP32 X."""
    pa, m, n, lda = colmajor(A)
    po, l, _, ldo = colmajor(Omega)
    X = empty_colmajor(l, n, torch.float32, A.device)
    px, _, _, ldx = colmajor(X)
    _check("rpid_sketch_fp8", lib().rpid_sketch_fp8(ctx.handle, pa, m, n, lda, po, l, ldo, px, ldx))
    return X


def rpid_select_columns(ctx: Context, X: torch.Tensor, k: int, sync: bool = True):
    """Column-wise LUPP on the sketch (Alg. 2, step 3).  Returns
    (J, Lf, Uf, diagU, k_eff, status); k_eff/status are None when sync=False."""
    px, l, n, ldx = colmajor(X)
    J = torch.empty(k, dtype=torch.int64, device=X.device)
    Lf = empty_colmajor(n, k, X.dtype, X.device)
    Uf = empty_colmajor(k, k, X.dtype, X.device)
    diag = torch.empty(k, dtype=X.dtype, device=X.device)
    keff = _I(-1)
    s = lib().rpid_select_columns(
        ctx.handle, px, dtype_code(X), l, n, ldx, k, J.data_ptr(), Lf.data_ptr(), Lf.stride(1),
        Uf.data_ptr(), Uf.stride(1), diag.data_ptr(), ctypes.byref(keff) if sync else None,
    )
    _check("rpid_select_columns", s, allow_positive=True)
    return J, Lf, Uf, diag, (keff.value if sync else None), (s if sync else None)


def rpid_select_columns_async(ctx: Context, X: torch.Tensor, k: int):
    """rpid_select_columns without the host read: returns (J, Lf, Uf, diagU,
    status) with status a device int64 tensor of one element (0, t + 1 for
    an exactly zero pivot at step t, or a negative RPID_ERR_* code), written
    in stream order."""
    px, l, n, ldx = colmajor(X)
    J = torch.empty(k, dtype=torch.int64, device=X.device)
    Lf = empty_colmajor(n, k, X.dtype, X.device)
    Uf = empty_colmajor(k, k, X.dtype, X.device)
    diag = torch.empty(k, dtype=X.dtype, device=X.device)
    status = torch.empty(1, dtype=torch.int64, device=X.device)
    _check("rpid_select_columns_async", lib().rpid_select_columns_async(
        ctx.handle, px, dtype_code(X), l, n, ldx, k, J.data_ptr(), Lf.data_ptr(), Lf.stride(1),
        Uf.data_ptr(), Uf.stride(1), diag.data_ptr(), status.data_ptr()))
    return J, Lf, Uf, diag, status


def rpid_sketch_sparse_sign(ctx: Context, A: torch.Tensor, rows: torch.Tensor, signs: torch.Tensor, l: int,
                            scale: float) -> torch.Tensor:
    """X = scale * S A with S the l x m sparse sign embedding given by rows
    (m x zeta int32) and signs (m x zeta int8), both contiguous on the device."""
    pa, m, n, lda = colmajor(A)
    if rows.dtype != torch.int32 or signs.dtype != torch.int8 or rows.shape != signs.shape or rows.shape[0] != m:
        raise ValueError("rows (int32) and signs (int8) must be m x zeta")
    rows, signs = rows.contiguous(), signs.contiguous()
    out_dtype = torch.float32 if A.dtype == torch.bfloat16 else A.dtype
    X = empty_colmajor(l, n, out_dtype, A.device)
    px, _, _, ldx = colmajor(X)
    s = lib().rpid_sketch_sparse_sign(ctx.handle, pa, dtype_code(A), m, n, lda, rows.data_ptr(), signs.data_ptr(),
                                      rows.shape[1], l, float(scale), px, dtype_code(X), ldx)
    _check("rpid_sketch_sparse_sign", s)
    return X


def rpid_sketch_srtt(ctx: Context, A: torch.Tensor, perm: torch.Tensor, phi: torch.Tensor,
                     sel: torch.Tensor) -> torch.Tensor:
    """X = Gamma A with the SRTT embedding given by perm (int32[m]), phi
    (int8[m]) and sel (int32[l]); BF16 A gives an FP32 X."""
    pa, m, n, lda = colmajor(A)
    if perm.dtype != torch.int32 or phi.dtype != torch.int8 or sel.dtype != torch.int32:
        raise ValueError("perm int32, phi int8, sel int32")
    if perm.numel() != m or phi.numel() != m:
        raise ValueError("perm and phi must have m entries")
    l = int(sel.numel())
    perm, phi, sel = perm.contiguous(), phi.contiguous(), sel.contiguous()
    out_dtype = torch.float32 if A.dtype == torch.bfloat16 else A.dtype
    X = empty_colmajor(l, n, out_dtype, A.device)
    px, _, _, ldx = colmajor(X)
    s = lib().rpid_sketch_srtt(ctx.handle, pa, dtype_code(A), m, n, lda, perm.data_ptr(), phi.data_ptr(),
                               sel.data_ptr(), l, px, dtype_code(X), ldx)
    _check("rpid_sketch_srtt", s)
    return X


class CSC:
    """A sparse m x n matrix in compressed sparse column form on the device
    (colptr int64[n+1], rowidx int64[nnz], vals float64 or float32)."""

    def __init__(self, colptr, rowidx, vals, m, n):
        self.colptr = colptr.to(torch.int64).contiguous()
        self.rowidx = rowidx.to(torch.int64).contiguous()
        self.vals = vals.contiguous()
        self.m, self.n = int(m), int(n)
        self.nnz = int(self.rowidx.numel())

    def args(self):
        return (self.colptr.data_ptr(), self.rowidx.data_ptr(), self.vals.data_ptr(), dtype_code(self.vals),
                self.m, self.n, self.nnz)


def rpid_sketch_csc(ctx: Context, A: CSC, Gamma: torch.Tensor) -> torch.Tensor:
    """X = Gamma A for a CSC matrix A; Gamma l x m of A's value type."""
    pg, l, m2, ldg = colmajor(Gamma)
    if m2 != A.m or Gamma.dtype != A.vals.dtype:
        raise ValueError("Gamma must be l x m with A's value type")
    X = empty_colmajor(l, A.n, A.vals.dtype, Gamma.device)
    px, _, _, ldx = colmajor(X)
    _check("rpid_sketch_csc", lib().rpid_sketch_csc(ctx.handle, *A.args(), pg, ldg, l, px, ldx))
    return X


def rpid_sketch_csc_sparse_sign(ctx: Context, A: CSC, rows: torch.Tensor, signs: torch.Tensor, l: int,
                                scale: float) -> torch.Tensor:
    """X = scale * S A for a CSC matrix A and a sparse sign embedding S."""
    if rows.dtype != torch.int32 or signs.dtype != torch.int8 or rows.shape != signs.shape or rows.shape[0] != A.m:
        raise ValueError("rows (int32) and signs (int8) must be m x zeta")
    rows, signs = rows.contiguous(), signs.contiguous()
    X = empty_colmajor(l, A.n, A.vals.dtype, A.vals.device)
    px, _, _, ldx = colmajor(X)
    s = lib().rpid_sketch_csc_sparse_sign(ctx.handle, *A.args(), rows.data_ptr(), signs.data_ptr(), rows.shape[1],
                                          l, float(scale), px, ldx)
    _check("rpid_sketch_csc_sparse_sign", s)
    return X


def rpid_csc_gather(ctx: Context, A: CSC, J=None) -> torch.Tensor:
    """Dense C = A(:, J) (m x k), or all of A when J is None."""
    k = A.n if J is None else int(J.numel())
    C = empty_colmajor(A.m, k, A.vals.dtype, A.vals.device)
    pc, _, _, ldc = colmajor(C)
    s = lib().rpid_csc_gather(ctx.handle, *A.args(), k, J.data_ptr() if J is not None else None, pc, ldc)
    _check("rpid_csc_gather", s)
    return C


def rpid_select_columns_cpqr(ctx: Context, X: torch.Tensor, k: int, sync: bool = True):
    """Column-pivoted Householder QR of the sketch, k steps (Rand-CPQR).
    Returns (J, Rf, diagR, k_eff, status); Rf is k x n in X's dtype."""
    px, l, n, ldx = colmajor(X)
    J = torch.empty(k, dtype=torch.int64, device=X.device)
    Rf = empty_colmajor(k, n, X.dtype, X.device)
    diag = torch.empty(k, dtype=X.dtype, device=X.device)
    keff = _I(-1)
    s = lib().rpid_select_columns_cpqr(ctx.handle, px, dtype_code(X), l, n, ldx, k, J.data_ptr(),
                                       Rf.data_ptr(), Rf.stride(1), diag.data_ptr(),
                                       ctypes.byref(keff) if sync else None)
    _check("rpid_select_columns_cpqr", s, allow_positive=True)
    return J, Rf, diag, (keff.value if sync else None), (s if sync else None)


def rpid_id_coeffs_cpqr(ctx, k, J, Rf):
    """Z = Rf(:, J)^{-1} Rf (k x n FP64)."""
    pr, k2, n, ldr = colmajor(Rf)
    Z = empty_colmajor(k, n, torch.float64, Rf.device)
    s = lib().rpid_id_coeffs_cpqr(ctx.handle, dtype_code(Rf), k, n, J.data_ptr(), pr, ldr, Z.data_ptr(),
                                  Z.stride(1))
    _check("rpid_id_coeffs_cpqr", s)
    return Z


def rpid_id_coeffs_ls(ctx, X, k, J):
    """Z = X(:, J)^+ X by least squares over all l rows (k x n FP64)."""
    px, l, n, ldx = colmajor(X)
    Z = empty_colmajor(k, n, torch.float64, X.device)
    _check("rpid_id_coeffs_ls", lib().rpid_id_coeffs_ls(ctx.handle, px, dtype_code(X), l, n, ldx, k, J.data_ptr(),
                                                        Z.data_ptr(), Z.stride(1)))
    return Z


def rpid_id_coeffs(ctx, X, k, J, Lf, Uf, refine_steps=0, want_eta=False):
    """Z (k x n, FP64) with Z(:, J) = I from the pivoted sketch (Sec. 4), and
    optionally Theorem 1's eta."""
    px, l, n, ldx = colmajor(X)
    Z = empty_colmajor(k, n, torch.float64, X.device)
    eta = ctypes.c_double(0.0)
    s = lib().rpid_id_coeffs(
        ctx.handle, px, dtype_code(X), l, n, ldx, k, J.data_ptr(), Lf.data_ptr(), Lf.stride(1),
        Uf.data_ptr(), Uf.stride(1), Z.data_ptr(), Z.stride(1), int(refine_steps),
        ctypes.byref(eta) if want_eta else None,
    )
    _check("rpid_id_coeffs", s)
    return Z, (eta.value if want_eta else None)


def rpid_cur(ctx, A, k, J):
    """Row skeleton I (LUPP on C = A(:, J)) and U = C^+ A R^+ (stable form).
    Returns (I, U, k_eff, status)."""
    pa, m, n, lda = colmajor(A)
    I = torch.empty(k, dtype=torch.int64, device=A.device)
    U = empty_colmajor(k, k, torch.float64, A.device)
    keff = _I(-1)
    s = lib().rpid_cur(ctx.handle, pa, dtype_code(A), m, n, lda, k, J.data_ptr(), I.data_ptr(),
                       U.data_ptr(), U.stride(1), ctypes.byref(keff))
    _check("rpid_cur", s, allow_positive=True)
    return I, U, keff.value, s


def rpid_residual(ctx, which, A, k, J, Z=None, I=None, U=None) -> float:
    """||A - C Z||_F / ||A||_F (which=RESIDUAL_ID), ||A - C U R||_F / ||A||_F
    (RESIDUAL_CUR) or ||A - Z^T R||_F / ||A||_F (RESIDUAL_ROW_ID, Z k x m)."""
    pa, m, n, lda = colmajor(A)
    out = ctypes.c_double(0.0)
    s = lib().rpid_residual(
        ctx.handle, int(which), pa, dtype_code(A), m, n, lda, k, J.data_ptr() if J is not None else None,
        Z.data_ptr() if Z is not None else None, Z.stride(1) if Z is not None else k,
        I.data_ptr() if I is not None else None,
        U.data_ptr() if U is not None else None, U.stride(1) if U is not None else k,
        ctypes.byref(out),
    )
    _check("rpid_residual", s)
    return out.value


def rpid_residual_sums(ctx, which, A, k, J, Z=None, I=None, U=None) -> torch.Tensor:
    """Device FP64 [||A - P Q||_F^2, ||A||_F^2] for the residual `which`, on
    the context's stream without synchronising."""
    pa, m, n, lda = colmajor(A)
    sums = torch.empty(2, dtype=torch.float64, device=A.device)
    s = lib().rpid_residual_sums(
        ctx.handle, int(which), pa, dtype_code(A), m, n, lda, k, J.data_ptr() if J is not None else None,
        Z.data_ptr() if Z is not None else None, Z.stride(1) if Z is not None else k,
        I.data_ptr() if I is not None else None,
        U.data_ptr() if U is not None else None, U.stride(1) if U is not None else k,
        sums.data_ptr(),
    )
    _check("rpid_residual_sums", s)
    return sums


def rpid_mlp_features(ctx, diagU, L, k_eff):
    f = torch.empty(L, dtype=torch.float32, device=diagU.device)
    _check("rpid_mlp_features",
           lib().rpid_mlp_features(ctx.handle, diagU.data_ptr(), dtype_code(diagU), L, k_eff, f.data_ptr()))
    return f


def rpid_mlp_forward(ctx, W, feats, want_act=True):
    B = feats.shape[0]
    y = torch.empty(B, dtype=torch.float32, device=feats.device)
    act = torch.empty((B, 2 * MLP_H), dtype=torch.float32, device=feats.device) if want_act else None
    _check("rpid_mlp_forward", lib().rpid_mlp_forward(
        ctx.handle, W.data_ptr(), feats.contiguous().data_ptr(), B, y.data_ptr(),
        act.data_ptr() if act is not None else None))
    return y, act


def rpid_mlp_backward(ctx, W, feats, act, dy):
    B = feats.shape[0]
    dW = torch.empty(MLP_NPARAM, dtype=torch.float32, device=feats.device)
    _check("rpid_mlp_backward", lib().rpid_mlp_backward(
        ctx.handle, W.data_ptr(), feats.contiguous().data_ptr(), act.data_ptr(),
        dy.contiguous().data_ptr(), B, dW.data_ptr()))
    return dW


def rpid_mlp_adam(ctx, W, dW, m1, m2, lr, t):
    _check("rpid_mlp_adam", lib().rpid_mlp_adam(
        ctx.handle, W.data_ptr(), dW.data_ptr(), m1.data_ptr(), m2.data_ptr(), float(lr), int(t)))


def rpid_mlp_loss(ctx, yhat, target, tau):
    """Pinball loss (device float tensor of one element) and its gradient dy."""
    B = yhat.shape[0]
    dy = torch.empty(B, dtype=torch.float32, device=yhat.device)
    loss = torch.empty(1, dtype=torch.float32, device=yhat.device)
    _check("rpid_mlp_loss", lib().rpid_mlp_loss(
        ctx.handle, yhat.contiguous().data_ptr(), target.contiguous().data_ptr(), B, float(tau),
        dy.data_ptr(), loss.data_ptr()))
    return loss, dy


class _SideWorker:
    """One thread that runs the side branch of decompose_overlapped, started
    once per side context and woken per step, so that no thread start sits
    between the column pivots and the CUR step's first launches."""

    def __init__(self):
        import threading

        self._go = threading.Event()
        self._done = threading.Event()
        self._job = None
        self._out = None
        self._pending = False  # a job started and its result not yet taken
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()

    def _loop(self):
        while True:
            self._go.wait()
            self._go.clear()
            job = self._job
            if job is None:
                return
            try:
                self._out = (job(), None)
            except Exception as e:  # noqa: BLE001 (re-raised in the caller's thread)
                self._out = (None, e)
            self._done.set()

    def start(self, job):
        self._job = job
        self._pending = True
        self._done.clear()
        self._go.set()

    def result(self):
        self._done.wait()
        self._pending = False
        out, err = self._out
        self._out = None
        if err is not None:
            raise err
        return out

    def stop(self):
        # a job already handed over runs to its end first: clearing it before
        # the thread has picked it up would drop it and leave result() waiting
        if self._pending:
            self._done.wait(timeout=60.0)
        self._job = None
        self._go.set()
        self._thread.join(timeout=5.0)


def _relative(sums: torch.Tensor) -> float:
    """||A - PQ||_F / ||A||_F from the device pair [||A - PQ||^2, ||A||^2]
    (the same expression the library evaluates for rpid_residual)."""
    d, a = sums.cpu().tolist()
    return math.sqrt(d / a) if a > 0.0 else 0.0


def decompose_overlapped(ctx, ctx2, A, Omega, k, refine_steps=None):
    """Alg. 2 end to end with both residuals, the two branches that follow
    the column pivots run concurrently: Z and the ID residual on ctx2's
    stream (enqueued by a worker thread that ctx2 keeps; the library calls
    release the interpreter lock), the CUR step and its residual on ctx's
    stream.  The CUR call is made as soon as the worker is woken, so its
    cooperative row LUPP launch finds the compute units free (the order that
    measured fastest); both residuals are left on the device
    (rpid_residual_sums) and read once at the end.  ctx2 needs its own
    stream; the two contexts have separate workspaces, so the branches share
    nothing but their read-only inputs.  The results are those of the
    sequential order (the same kernels on the same inputs)."""
    X = rpid_sketch(ctx, A, Omega)
    if refine_steps is None:
        refine_steps = 0 if X.dtype == torch.float64 else 1
    # the pivots' status is read before the branches are enqueued: with it
    # left on the device (rpid_select_columns_async) the side branch's first
    # kernels reach the compute units together with the row LUPP, whose
    # cooperative launch then waits for them (measured slower)
    J, Lf, Uf, diag, keff, st = rpid_select_columns(ctx, X, k)
    out = dict(X=X, J=J, Lf=Lf, Uf=Uf, diag=diag, k_eff=keff, status=st)
    if st != 0:
        return out
    worker = ctx2.__dict__.get("_side_worker")
    if worker is None:
        worker = ctx2._side_worker = _SideWorker()
    ready = torch.cuda.Event()
    ready.record(ctx.stream)

    def id_branch():
        ctx2.stream.wait_event(ready)
        Z, _ = rpid_id_coeffs(ctx2, X, k, J, Lf, Uf, refine_steps=refine_steps)
        return Z, rpid_residual_sums(ctx2, RESIDUAL_ID, A, k, J, Z=Z)

    worker.start(id_branch)
    try:
        I, U, keff_i, st_i = rpid_cur(ctx, A, k, J)
        scur = rpid_residual_sums(ctx, RESIDUAL_CUR, A, k, J, I=I, U=U) if st_i == 0 else None
    finally:
        # also when the CUR branch raised: the side stream may still be
        # writing Z and its sums, which must not be freed before it is done
        try:
            Z, sid = worker.result()
        finally:
            ctx2.stream.synchronize()
    ctx.stream.synchronize()
    out.update(Z=Z, I=I, U=U, status_I=st_i, residual_id=_relative(sid),
               residual_cur=_relative(scur) if scur is not None else None)
    return out


def decompose(ctx, A, Omega, k, refine_steps=None, want_eta=False, want_cur=True):
    """The whole path: sketch, column LUPP, Z, and (optionally) CUR.  The
    LUPP runs in FP64 for FP64 storage and in FP32 otherwise."""
    X = rpid_sketch(ctx, A, Omega)
    if refine_steps is None:
        refine_steps = 0 if X.dtype == torch.float64 else 1
    J, Lf, Uf, diag, keff, st = rpid_select_columns(ctx, X, k)
    out = dict(X=X, J=J, Lf=Lf, Uf=Uf, diag=diag, k_eff=keff, status=st)
    if st != 0:
        return out
    Z, eta = rpid_id_coeffs(ctx, X, k, J, Lf, Uf, refine_steps=refine_steps, want_eta=want_eta)
    out.update(Z=Z, eta=eta)
    if want_cur:
        I, U, keff_i, st_i = rpid_cur(ctx, A, k, J)
        out.update(I=I, U=U, status_I=st_i)
    return out
