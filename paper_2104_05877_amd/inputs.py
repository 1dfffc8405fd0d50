"""Seeded synthetic inputs for randomized LUPP skeleton selection.

This module only builds test matrices and Gaussian embeddings; it holds none
of the method's arithmetic.  Both the FP64 oracle (through the tests) and the
HIP path take their inputs from here, so the two see identical values.

Matrices are returned column-major: a numpy array in Fortran order, or a torch
tensor ``t`` whose transpose ``t.T`` is contiguous (``t.stride() == (1, m)``).

Workload recipes (the paper's own datasets are not used; these synthetic
matrices stand in for them, with spectra controlled exactly):

* ``spectral``: A = U diag(s) V^T with U, V Haar-distributed orthonormal
  factors (QR of a Gaussian matrix with the sign of diag(R) folded in).
* ``lowrank_noise``: A = F G + sigma N, F, G Gaussian factors.
* ``nonneg_lowrank``: A = |F| |G| + uniform noise (non-negative entries).
* ``gaussian_embedding``: Omega with iid N(0, 1) entries (the embedding of
  Section 2.2 with mean 0; the scale does not change the pivots).
* ``sparse_sign_draws``: the random draws of a sparse sign embedding (Section
  2.2): for each of its m columns, zeta distinct row coordinates uniform over
  the l rows and zeta independent signs.
* ``srtt_draws``: the random draws of an SRTT embedding (Section 2.2): a
  permutation of the m rows, m Rademacher signs and l distinct rows of the
  m x m transform.
* ``snn_csc``: a sparse non-negative (SNN) matrix sum_i s_i x_i y_i^T with
  sparse non-negative x_i, y_i (eq. snn-def), in compressed sparse column
  form.  The paper leaves the sparsity of x_i, y_i open: here each x_i
  (y_i) has round(rho m) (round(rho n)) nonzeros at uniform positions with
  values uniform on (0, 1).
"""
from __future__ import annotations

import numpy as np

# Workload shapes: (m, n, k, l).
WORKLOADS = {
    "exp1000x800": dict(m=1000, n=800, k=50, l=50),
    "poly8192": dict(m=8192, n=8192, k=256, l=272),
    "lowrank16384_bf16": dict(m=16384, n=16384, k=512, l=544),
    "nonneg65536x4096_fp8": dict(m=65536, n=4096, k=384, l=400),
}

STREAM_U, STREAM_V, STREAM_OMEGA, STREAM_NOISE = 0, 1, 2, 3


def rng_for(case: int, rep: int, stream: int) -> np.random.Generator:
    """Independent PCG64 stream for (case, repetition, stream)."""
    return np.random.default_rng([1000 * case + rep, stream])


def haar(rng: np.random.Generator, m: int, r: int) -> np.ndarray:
    """m x r matrix with orthonormal columns, Haar distributed (Mezzadri)."""
    g = rng.standard_normal((m, r))
    q, rr = np.linalg.qr(g)
    d = np.sign(np.diag(rr))
    d[d == 0] = 1.0
    return q * d


def spectral(m: int, n: int, s: np.ndarray, rng_u, rng_v) -> np.ndarray:
    """A = U diag(s) V^T, float64, Fortran order; len(s) <= min(m, n)."""
    s = np.asarray(s, dtype=np.float64)
    r = s.shape[0]
    u = haar(rng_u, m, r)
    v = haar(rng_v, n, r)
    return np.asfortranarray((u * s) @ v.T)


def exp_spectrum(r: int, decades: float = 8.0) -> np.ndarray:
    """s_i = 10^(-decades (i-1)/(r-1)), i = 1..r."""
    i = np.arange(r, dtype=np.float64)
    return 10.0 ** (-decades * i / (r - 1))


def poly_spectrum(r: int, power: float = 2.0) -> np.ndarray:
    """s_i = i^(-power), i = 1..r."""
    return np.arange(1, r + 1, dtype=np.float64) ** (-power)


def gaussian_embedding(rng: np.random.Generator, l: int, m: int) -> np.ndarray:
    """l x m iid N(0, 1), float64, Fortran order."""
    return np.asfortranarray(rng.standard_normal((l, m)))


def lowrank_noise(rng_f, rng_g, rng_e, m, n, r, noise) -> np.ndarray:
    """F (m x r) G (r x n) + noise * N(0,1), float64, Fortran order."""
    f = rng_f.standard_normal((m, r))
    g = rng_g.standard_normal((r, n))
    a = f @ g
    a += noise * rng_e.standard_normal((m, n))
    return np.asfortranarray(a)


def nonneg_lowrank(rng_f, rng_g, rng_e, m, n, r, noise) -> np.ndarray:
    """|F| |G| + uniform[0, noise], float64, Fortran order."""
    f = np.abs(rng_f.standard_normal((m, r)))
    g = np.abs(rng_g.standard_normal((r, n)))
    a = f @ g
    a += noise * rng_e.random((m, n))
    return np.asfortranarray(a)


def case_exp1000x800(rep: int = 0):
    """1000 x 800, Haar U (1000 x 800) and V (800 x 800), exponential
    spectrum over 8 decades; k = l = 50; Omega 50 x 1000 N(0, 1)."""
    w = WORKLOADS["exp1000x800"]
    s = exp_spectrum(800, 8.0)
    a = spectral(w["m"], w["n"], s, rng_for(0, rep, STREAM_U), rng_for(0, rep, STREAM_V))
    om = gaussian_embedding(rng_for(0, rep, STREAM_OMEGA), w["l"], w["m"])
    return a, om, w["k"], w["l"]


def small_spectral_case(m, n, k, l, s, seed):
    """Any small spectral case: (A, Omega) float64 Fortran order."""
    a = spectral(m, n, s, rng_for(seed, 0, STREAM_U), rng_for(seed, 0, STREAM_V))
    om = gaussian_embedding(rng_for(seed, 0, STREAM_OMEGA), l, m)
    return a, om


# --------------------------------------------------------------------------
# Device-side generation (torch) for the large workloads.  Values come from
# torch's own generator; the oracle receives the very same values by copying
# the generated tensors back to the host.
# --------------------------------------------------------------------------
def _torch():
    import torch  # noqa: PLC0415

    return torch


def torch_colmajor(a_np, dtype, device):
    """Copy a Fortran-order numpy matrix into a column-major torch tensor."""
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a_np).T)).to(device=device, dtype=dtype)
    return t.T


def empty_colmajor(rows, cols, dtype, device):
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype, device=device).T


def torch_haar(gen, m, r, device):
    torch = _torch()
    g = torch.randn((m, r), generator=gen, dtype=torch.float64, device=device)
    q, rr = torch.linalg.qr(g)
    d = torch.sign(torch.diagonal(rr))
    d[d == 0] = 1.0
    return q * d


def torch_spectral(m, n, s, seed, device):
    """A = U diag(s) V^T in float64 on ``device``, column-major."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    s_t = torch.as_tensor(np.asarray(s, dtype=np.float64), device=device)
    r = s_t.shape[0]
    u = torch_haar(gen, m, r, device)
    v = torch_haar(gen, n, r, device)
    # column-major result: build A^T (n x m) contiguous, return its transpose
    at = (v * s_t) @ u.T
    return at.T


def torch_poly8192(seed, device, m=8192, n=8192, l=272):
    """The 8192 x 8192 benchmark workload: A = U diag(s) V^T with Haar U, V
    and s_i = i^-2, generated in float64 and stored float32, and a Gaussian
    embedding Omega (l x m) stored float32.  Returns (A32, Omega32),
    column-major on ``device``."""
    torch = _torch()
    a64 = torch_spectral(m, n, poly_spectrum(min(m, n), 2.0), seed, device)
    a32 = a64.T.contiguous().float().T
    del a64
    om32 = torch_gaussian(l, m, seed + 7, device).T.contiguous().float().T
    return a32, om32


def torch_gaussian(rows, cols, seed, device, dtype=None):
    """rows x cols iid N(0,1), column-major, float64 unless dtype given."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    t = torch.randn((cols, rows), generator=gen, dtype=torch.float64, device=device)
    if dtype is not None:
        t = t.to(dtype)
    return t.T


def torch_lowrank_noise(m, n, r, noise, seed, device):
    """F G + noise N(0,1) in float32, column-major (rank-r Gaussian factors)."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f = torch.randn((m, r), generator=gen, dtype=torch.float32, device=device)
    g = torch.randn((r, n), generator=gen, dtype=torch.float32, device=device)
    at = (f @ g).T.contiguous()
    at += noise * torch.randn((n, m), generator=gen, dtype=torch.float32, device=device)
    return at.T


def torch_nonneg_lowrank(m, n, r, noise, seed, device):
    """|F| |G| + uniform[0, noise] in float32, column-major."""
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f = torch.randn((m, r), generator=gen, dtype=torch.float32, device=device).abs_()
    g = torch.randn((r, n), generator=gen, dtype=torch.float32, device=device).abs_()
    at = (f @ g).T.contiguous()
    at += noise * torch.rand((n, m), generator=gen, dtype=torch.float32, device=device)
    return at.T


# ---------------------------------------------------------------------------
# learned-rank stream: matrices drawn per index from a seed-chosen mix of
# exponential and polynomial spectral decays
# ---------------------------------------------------------------------------
def stream_spec(index, seed=0, m_range=(2048, 8192), n_range=(2048, 8192),
                rate_range=(1e-3, 1e-1), power_range=(0.5, 3.0), floor=1e-12):
    """(m, n, spectrum, family) of matrix `index` of a stream: m, n uniform
    integers in their ranges; with probability 1/2 s_i = exp(-rate (i-1)) with
    rate log-uniform, else s_i = i^-power with power uniform; truncated where
    s_i / s_1 < floor."""
    rng = rng_for(40 + seed, index, STREAM_NOISE)
    m = int(rng.integers(m_range[0], m_range[1] + 1))
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    r = min(m, n)
    i = np.arange(r, dtype=np.float64)
    if rng.random() < 0.5:
        rate = float(np.exp(rng.uniform(np.log(rate_range[0]), np.log(rate_range[1]))))
        spec, fam = np.exp(-rate * i), ("exp", rate)
    else:
        power = float(rng.uniform(power_range[0], power_range[1]))
        spec, fam = (i + 1.0) ** (-power), ("poly", power)
    spec = spec[spec >= floor * spec[0]]
    return m, n, spec, fam


def torch_stream_case(index, lmax, device, seed=0, with_lo=True, **ranges):
    """Matrix `index` of the stream on the GPU: (A64, Omega64 (lmax x m),
    A_bf16, Omega_bf16, family), column-major (the BF16 copies are None when
    with_lo is false)."""
    torch = _torch()
    m, n, spec, fam = stream_spec(index, seed, **ranges)
    a64 = torch_spectral(m, n, spec, 100003 * (seed + 1) + 7 * index, device)
    om64 = torch_gaussian(lmax, m, 200003 * (seed + 1) + 11 * index, device)
    if not with_lo:
        return a64, om64, None, None, fam
    a16 = a64.T.contiguous().bfloat16().T
    om16 = om64.T.contiguous().bfloat16().T
    return a64, om64, a16, om16, fam


def sparse_sign_draws(rng: np.random.Generator, m: int, l: int, zeta: int):
    """rows (m x zeta int32) and signs (m x zeta int8): column i of the
    embedding has the value signs[i, s] at row rows[i, s], s < zeta; the rows
    of a column are distinct and uniform (the first zeta of a random
    permutation of the l rows), the signs independent Rademacher."""
    keys = rng.random((m, l))
    rows = np.argpartition(keys, zeta - 1, axis=1)[:, :zeta].astype(np.int32)
    signs = np.where(rng.random((m, zeta)) < 0.5, -1, 1).astype(np.int8)
    return np.ascontiguousarray(rows), np.ascontiguousarray(signs)


def snn_csc(rng: np.random.Generator, m: int, n: int, s: np.ndarray, rho: float):
    """SNN matrix sum_i s_i x_i y_i^T (eq. snn-def) as (colptr int64[n+1],
    rowidx int64[nnz], vals float64[nnz]) with sorted row indices per
    column; x_i, y_i have round(rho m), round(rho n) nonzeros (at least 1)
    at uniform positions, values uniform on (0, 1)."""
    r = len(s)
    px = max(1, int(round(rho * m)))
    py = max(1, int(round(rho * n)))
    cols = {}
    for i in range(r):
        xi = rng.choice(m, px, replace=False)
        xv = rng.random(px)
        yi = rng.choice(n, py, replace=False)
        yv = rng.random(py)
        for jj, yy in zip(yi, yv):
            d = cols.setdefault(int(jj), {})
            w = s[i] * yy
            for ii, xx in zip(xi, xv):
                d[int(ii)] = d.get(int(ii), 0.0) + w * xx
    colptr = np.zeros(n + 1, dtype=np.int64)
    rowidx, vals = [], []
    for j in range(n):
        d = cols.get(j, {})
        keys = sorted(d)
        rowidx.extend(keys)
        vals.extend(d[k] for k in keys)
        colptr[j + 1] = colptr[j] + len(keys)
    return colptr, np.array(rowidx, dtype=np.int64), np.array(vals, dtype=np.float64)


def srtt_draws(rng: np.random.Generator, m: int, l: int):
    """perm (int32[m], a uniform permutation), phi (int8[m], +-1) and sel
    (int32[l], l distinct rows out of m, uniform)."""
    perm = rng.permutation(m).astype(np.int32)
    phi = np.where(rng.random(m) < 0.5, -1, 1).astype(np.int8)
    sel = rng.choice(m, l, replace=False).astype(np.int32)
    return perm, phi, sel
