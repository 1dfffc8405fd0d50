"""Pins of the fixed-arithmetic LUPP oracle (oracle/lupp_fma.c, reached through
oracle.rpid_oracle.lupp_colwise_fma).

Its arithmetic is pinned by an independent emulation in exact rational
arithmetic with one explicit rounding per division and per fused update
(every value on tiny panels, float64 and float32); its pivots by LAPACK's
getrf on tie-free inputs, Lemma 2's worked example, the greedy maximal-volume
property and the tie/zero-pivot rules.  Planted mistakes in a copy of the C
source are caught by these pins.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import oracle.rpid_oracle as O
from tests.oracle_pins import kahan_matrix, load_kahan_golden


# ---------------------------------------------------------------------------
# exact rounding of a rational to binary64 / binary32 (nearest, ties to even)
# ---------------------------------------------------------------------------
def _round_to(fr: Fraction, mant_bits: int) -> Fraction:
    if fr == 0:
        return Fraction(0)
    sign = -1 if fr < 0 else 1
    a = abs(fr)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    # a in [2^e, 2^(e+1)); keep mant_bits significant bits
    scale = Fraction(2) ** (e - (mant_bits - 1))
    q = a / scale
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return sign * n * scale


def _rnd(fr, dtype):
    return _round_to(fr, 53 if dtype == np.float64 else 24)


def exact_lupp(S, k, dtype):
    """LUPP of the n x k panel S with every division and every fused update
    rounded once from its exact rational value."""
    S = [[Fraction(float(v)) for v in row] for row in S]
    n = len(S)
    done = [False] * n
    J = []
    L = [[Fraction(0)] * k for _ in range(n)]
    U = [[Fraction(0)] * k for _ in range(k)]
    for t in range(k):
        p, best = -1, Fraction(-1)
        for i in range(n):
            if not done[i] and abs(S[i][t]) > best:
                best, p = abs(S[i][t]), i
        if best == 0:
            break
        J.append(p)
        for c in range(t, k):
            U[t][c] = S[p][c]
        done[p] = True
        L[p][t] = Fraction(1)
        for i in range(n):
            if done[i]:
                continue
            m = _rnd(S[i][t] / S[p][t], dtype)
            L[i][t] = m
            for c in range(t + 1, k):
                S[i][c] = _rnd(S[i][c] - m * U[t][c], dtype)
    return (np.array(J, dtype=np.int64), np.array([[float(v) for v in r] for r in L]),
            np.array([[float(v) for v in r] for r in U]))


def _check_exact(lupp, dtype, seeds=range(6), n=7, k=4):
    for seed in seeds:
        rng = np.random.default_rng(seed)
        X = rng.standard_normal((k, n)).astype(dtype)
        f = lupp(X, k, dtype)
        J, L, U = exact_lupp(X.T.astype(np.float64), k, dtype)
        assert np.array_equal(f["J"], J), (seed, f["J"], J)
        assert np.array_equal(f["L"].astype(np.float64), L), seed
        assert np.array_equal(f["U"].astype(np.float64), U), seed


def pin_exact_arithmetic(lupp):
    """Every value equals the exact-rational emulation with one rounding per
    division and per fused update (float64 and float32)."""
    _check_exact(lupp, np.float64)
    _check_exact(lupp, np.float32)


def pin_getrf(lupp):
    """Pivots equal LAPACK getrf's on tie-free inputs; L and U agree to
    rounding (float64 and float32 data)."""
    for dtype, tol in ((np.float64, 1e-11), (np.float32, 2e-4)):
        rng = np.random.default_rng(5)
        X = rng.standard_normal((12, 40)).astype(dtype)
        f = lupp(X, 12, dtype)
        lu, piv = sla.lu_factor(X.astype(np.float64).T)
        perm = np.arange(40)
        for t, p in enumerate(piv[:12]):
            perm[t], perm[p] = perm[p], perm[t]
        assert np.array_equal(f["J"], perm[:12])
        Lr = np.tril(lu[:, :12], -1)[np.argsort(perm)] + 0.0
        Lr[perm[:12], np.arange(12)] = 1.0
        assert np.abs(f["L"].astype(np.float64) - Lr).max() <= tol
        assert np.abs(f["U"].astype(np.float64) - np.triu(lu[:12, :12])).max() <= tol * 10


def pin_kahan_exact(lupp):
    """Lemma 2's worked example: every candidate ties, J = 0..l-1, and the
    factors are exact (small integers) in either precision."""
    for l, n, _ in load_kahan_golden():
        X = kahan_matrix(l, n)
        for dtype in (np.float64, np.float32):
            f = lupp(X, l, dtype)
            assert np.array_equal(f["J"], np.arange(l))
            # U(t, :) is column t of R_1 from the diagonal on: the identity;
            # the multipliers are R_1^T (-1 below the unit diagonal) for the
            # first l columns and 1 for every all-ones column of R_2
            assert np.array_equal(f["U"].astype(np.float64), np.eye(l))
            L = f["L"].astype(np.float64)
            assert np.array_equal(L[:l], X[:, :l].T)
            assert np.all(L[l:] == 1.0)


def pin_greedy_volume(lupp, seed=11, l=5, n=9):
    """Each pivot maximises |det X(0:t+1, J_<t + [j])| over remaining j."""
    X = np.random.default_rng(seed).standard_normal((l, n))
    J = list(lupp(X, l, np.float64)["J"])
    for t in range(l):
        dets = {j: abs(np.linalg.det(X[: t + 1, J[:t] + [j]])) for j in range(n) if j not in J[:t]}
        assert J[t] == max(dets, key=lambda j: (dets[j], -j)), t


def pin_ties_and_zero(lupp):
    """Equal moduli go to the smallest column; an exactly zero pivot stops
    with status t + 1; a NaN is rejected."""
    X = np.array([[1.0, -2.0, 2.0, 0.5], [3.0, 1.0, 1.0, 0.0]])
    f = lupp(X, 2, np.float64)
    assert f["J"][0] == 1  # |-2| ties with |2|: the smaller column wins
    Z = np.array([[4.0, 2.0, 1.0, 0.0], [0.0, 2.0, 1.0, 1.0], [4.0, 4.0, 2.0, 1.0]])
    g = lupp(Z, 3, np.float64)
    assert g["status"] == 3 and g["k_eff"] == 2 and list(g["J"]) == [0, 1]
    Xn = np.ones((3, 5))
    Xn[1, 2] = np.nan
    with pytest.raises(O.NonFiniteInput):
        lupp(Xn, 3, np.float64)


PINS = [pin_exact_arithmetic, pin_getrf, pin_kahan_exact, pin_greedy_volume, pin_ties_and_zero]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_fma_pin(pin):
    pin(O.lupp_colwise_fma)


def test_fma_pivots_match_numpy_oracle():
    """Where no two candidates come within rounding of each other, the fused
    and the unfused oracle pick the same pivots."""
    X = np.random.default_rng(3).standard_normal((64, 3000))
    a = O.lupp_colwise(X, 64, gaps=True)
    b = O.lupp_colwise_fma(X, 64)
    assert a["gap"].min() > 1e-9
    assert np.array_equal(a["J"], b["J"])
    assert np.abs(a["U"] - b["U"]).max() <= 1e-12 * np.abs(a["U"]).max()


# ---------------------------------------------------------------------------
# planted mistakes in a copy of the C source must be caught by some pin
# ---------------------------------------------------------------------------
C_MUTANTS = {
    "unfused update": ("S[i * k + c] = FMA(-m, U[t * k + c], S[i * k + c]);",
                       "S[i * k + c] = S[i * k + c] - m * U[t * k + c];"),
    "reciprocal instead of division": ("const T m = S[i * k + t] / piv;",
                                       "const T m = S[i * k + t] * ((T)1 / piv);"),
    "ties to the larger column": ("if (a > best) {", "if (a >= best) {"),
    "update sign": ("FMA(-m, U[t * k + c], S[i * k + c])", "FMA(m, U[t * k + c], S[i * k + c])"),
    "argmax without the modulus": ("T a = FABS(S[i * k + t]);", "T a = S[i * k + t];"),
}


def _mutant_lupp(tmp_path, name, old, new):
    src = open(O.FMA_SRC).read()
    assert old in src, name
    path = tmp_path / ("m_%d.c" % abs(hash(name)))
    path.write_text(src.replace(old, new))
    so = str(path) + ".so"
    subprocess.run(["gcc", *O.FMA_CFLAGS, str(path), "-o", so, "-lm"], check=True, capture_output=True)
    lib = ctypes.CDLL(so)
    P = ctypes.c_void_p
    for fn in ("lupp_fma_f64", "lupp_fma_f32"):
        getattr(lib, fn).restype = ctypes.c_int
        getattr(lib, fn).argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, P, P]

    def lupp(X, k, dtype=np.float64):
        saved = O._FMA_LIB
        O._FMA_LIB = lib
        try:
            return O.lupp_colwise_fma(X, k, dtype)
        finally:
            O._FMA_LIB = saved

    return lupp


@pytest.mark.parametrize("name", list(C_MUTANTS))
def test_fma_mutant_caught(tmp_path, name):
    lupp = _mutant_lupp(tmp_path, name, *C_MUTANTS[name])
    caught = []
    for pin in PINS:
        try:
            pin(lupp)
        except (AssertionError, ValueError, O.NonFiniteInput, IndexError):
            caught.append(pin.__name__)
    assert caught, name
