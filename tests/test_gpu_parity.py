"""GPU path (through the C-ABI) against the FP64 oracle, element by element.

Pivot vectors must be bit-exact in FP64 arithmetic; floating-point results
are compared within tolerances derived in the test from the arithmetic.
Cases span several tiles and ragged tails; each prints what it runs first.
"""
import sys

import numpy as np
import pytest

import oracle.rpid_oracle as O
from paper_2104_05877_amd import inputs
from tests.oracle_pins import kahan_matrix, load_kahan_golden

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    from paper_2104_05877_amd import rpid

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return rpid


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


def dev(a_np, dtype=torch.float64):
    return inputs.torch_colmajor(a_np, dtype, "cuda")


def host(t):
    return t.detach().double().cpu().numpy()


# ---------------------------------------------------------------------------
# LUPP (select_columns)
# ---------------------------------------------------------------------------
def test_lupp_kahan_golden(R, ctx):
    """Lemma 2's worked example: every candidate ties at |1|; the GPU must keep
    J = 0..l-1 (smallest-index rule across workgroups) and reproduce
    Z_rest(i, :) = 2^(l-1-i) exactly."""
    for l, n, rowvals in load_kahan_golden():
        say("kahan", l, n)
        X = dev(kahan_matrix(l, n))
        J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, X, l)
        assert st == 0 and keff == l
        assert host(J).astype(np.int64).tolist() == list(range(l))
        Z, eta = R.rpid_id_coeffs(ctx, X, l, J, Lf, Uf, want_eta=True)
        zr = host(Z)[:, l:]
        assert np.array_equal(zr, np.repeat(rowvals[:, None], n - l, axis=1))
        ref = np.sqrt(1.0 + (n - l) * (4.0**l - 1.0) / 3.0)
        assert abs(eta - ref) <= 1e-9 * ref


def test_lupp_ties_across_workgroups(R, ctx):
    """Duplicated columns spread over many workgroups: ties resolve to the
    smallest column index, as in the oracle."""
    say("ties", 6, 3000)
    rng = np.random.default_rng(1)
    base = rng.standard_normal((6, 40))
    X = np.tile(base, (1, 75))  # column j equals column j mod 40
    f = O.lupp_colwise(X, 6)
    J, *_ , keff, st = R.rpid_select_columns(ctx, dev(X), 6)
    assert st == 0
    assert np.array_equal(host(J).astype(np.int64), f["J"])


@pytest.mark.parametrize("l,n,k,seed", [(40, 1000, 40, 1), (64, 3001, 37, 2), (300, 2500, 256, 3),
                                        (20, 20, 20, 4), (8, 100, 1, 5), (520, 5000, 512, 6)])
def test_lupp_f64_parity(R, ctx, l, n, k, seed):
    """FP64 LUPP on a seeded Gaussian sketch: pivots bit-exact; multipliers
    and U within a few ulps of the oracle times the growth."""
    say("lupp_f64", l, n, k, seed)
    X = np.random.default_rng(seed).standard_normal((l, n))
    f = O.lupp_colwise(X, k, gaps=True)
    assert f["gap"].min() > 1e-9  # no near-tie: the pivots are unique
    J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, dev(X), k)
    assert st == 0 and keff == k
    assert np.array_equal(host(J).astype(np.int64), f["J"])
    tol = 1e-11 * max(1.0, np.abs(f["U"]).max())
    np.testing.assert_allclose(host(Lf), f["L"], rtol=0, atol=1e-11)
    np.testing.assert_allclose(host(Uf), f["U"], rtol=0, atol=tol)
    np.testing.assert_allclose(host(diag), f["diag"], rtol=0, atol=tol)


def test_lupp_f64_largest_k(R, ctx):
    """The largest k the boundary accepts (k = l = 1024; 2048 candidates):
    FP64 pivots bit-exact, factors within the same tolerances."""
    l = n_l = 1024
    n, k = 2048, 1024
    say("lupp_f64 largest k", l, n, k)
    X = np.random.default_rng(9).standard_normal((l, n))
    f = O.lupp_colwise(X, k, gaps=True)
    assert f["gap"].min() > 1e-9 and n_l == k
    J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, dev(X), k)
    assert st == 0 and keff == k
    assert np.array_equal(host(J).astype(np.int64), f["J"])
    tol = 1e-11 * max(1.0, np.abs(f["U"]).max())
    np.testing.assert_allclose(host(Lf), f["L"], rtol=0, atol=1e-10)
    np.testing.assert_allclose(host(Uf), f["U"], rtol=0, atol=tol)
    with pytest.raises(R.RpidError):
        R.rpid_select_columns(ctx, dev(np.ones((1100, 2048))), 1025)


@pytest.mark.parametrize("l,n,k,seed", [(40, 2000, 40, 7), (272, 8192, 256, 8)])
def test_lupp_f32_parity(R, ctx, l, n, k, seed):
    """FP32 LUPP on FP32-representable data; the oracle runs in FP64 on the
    same values.  Where the oracle's relative pivot gap exceeds 1e-3 (far above
    FP32 rounding of the Schur complements here) the pivots must agree."""
    say("lupp_f32", l, n, k, seed)
    X = np.random.default_rng(seed).standard_normal((l, n)).astype(np.float32).astype(np.float64)
    f = O.lupp_colwise(X, k, gaps=True)
    J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, dev(X, torch.float32), k)
    assert st == 0
    Jg = host(J).astype(np.int64)
    first_close = np.argmax(f["gap"] < 1e-3) if (f["gap"] < 1e-3).any() else k
    assert np.array_equal(Jg[:first_close], f["J"][:first_close])
    if first_close == k:
        np.testing.assert_allclose(host(Lf), f["L"], rtol=0, atol=5e-4)


def test_lupp_zero_pivot_and_nonfinite(R, ctx):
    """Exactly rank-deficient sketch: status = step + 1 of the zero pivot;
    a NaN in the panel is reported, not pivoted on."""
    say("zero pivot")
    X = np.array([[4.0, 2.0, 1.0, 0.0], [0.0, 2.0, 1.0, 1.0], [4.0, 4.0, 2.0, 1.0]])
    J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, dev(X), 3)
    assert st == 3 and keff == 2
    assert host(J)[:2].astype(np.int64).tolist() == [0, 1]
    say("nonfinite")
    Xn = np.random.default_rng(3).standard_normal((8, 300))
    Xn[5, 200] = np.nan
    with pytest.raises(R.RpidError) as e:
        R.rpid_select_columns(ctx, dev(Xn), 8)
    assert e.value.status == -100


# ---------------------------------------------------------------------------
# Sketch
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,l,seed", [(1000, 800, 50, 1), (777, 1234, 300, 2), (4099, 513, 17, 3),
                                        (8192, 1024, 272, 4), (64, 3000, 1024, 5)])
def test_sketch_f64(R, ctx, m, n, l, seed):
    """FP64 MFMA sketch vs numpy: |X - X_ref| <= 8 sqrt(m) u |Omega| |A| (a
    bound on the rounding of any summation order)."""
    say("sketch_f64", m, n, l)
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    Om = rng.standard_normal((l, m))
    X = host(R.rpid_sketch(ctx, dev(A), dev(Om)))
    ref = O.sketch(A, Om)
    bound = 8 * np.sqrt(m) * 2.0**-53 * (np.abs(Om) @ np.abs(A))
    assert np.all(np.abs(X - ref) <= bound)


@pytest.mark.parametrize("m,n,l,seed", [(1000, 800, 50, 1), (4099, 515, 272, 2), (512, 700, 544, 3)])
def test_sketch_f32_bf16(R, ctx, m, n, l, seed):
    """FP32 (FP32 MFMA) and BF16 (BF16 MFMA, FP32 accumulation) sketches vs
    the FP64 sketch of the same stored values: error within the FP32
    accumulation bound 2 m u32 |Omega| |A|."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    Om = rng.standard_normal((l, m))
    for dt in (torch.float32, torch.bfloat16):
        say("sketch", dt, m, n, l)
        Ad, Od = dev(A, dt), dev(Om, dt)
        X = host(R.rpid_sketch(ctx, Ad, Od))
        a_s, o_s = host(Ad), host(Od)
        ref = O.sketch(a_s, o_s)
        bound = 2 * m * 2.0**-24 * (np.abs(o_s) @ np.abs(a_s))
        assert np.all(np.abs(X - ref) <= bound), dt


@pytest.mark.parametrize("m,n,l,seed", [(2048, 1000, 272, 6), (8192, 515, 300, 7), (1024, 130, 5, 8),
                                        (4096, 2048, 544, 9), (256, 64, 16, 10), (16384, 200, 400, 11)])
def test_sketch_stream_kernel(R, ctx, m, n, l, seed):
    """Sizes that take the streaming kernel (K a whole number of 256-byte
    stage pairs): row tiles of 1, 10, 13 and 17 with rows past l, ragged
    column strips, one and several K-ranges, two l-chunks.  FP32 and BF16
    against the FP64 product of the stored values, within the FP32
    accumulation bound."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    Om = rng.standard_normal((l, m))
    for dt in (torch.float32, torch.bfloat16):
        say("sketch stream", dt, m, n, l)
        Ad, Od = dev(A, dt), dev(Om, dt)
        X = host(R.rpid_sketch(ctx, Ad, Od))
        a_s, o_s = host(Ad), host(Od)
        ref = O.sketch(a_s, o_s)
        bound = 2 * m * 2.0**-24 * (np.abs(o_s) @ np.abs(a_s))
        assert np.all(np.abs(X - ref) <= bound), dt


# ---------------------------------------------------------------------------
# The whole path in FP64 on the 1000 x 800 exponential-spectrum workload
# ---------------------------------------------------------------------------
def test_exp1000x800_f64_end_to_end(R, ctx):
    """Sketch, LUPP, Z, CUR, residuals on GPU vs the oracle: J and I
    bit-exact, Z and U within conditioning-derived tolerances, residuals
    within 1e-9 relative, eta within 1e-6."""
    say("exp1000x800 f64")
    A, Om, k, l = inputs.case_exp1000x800()
    o = O.decompose(A, Om, k, gaps=True)
    assert o["gap_J"].min() > 1e-6 and o["gap_I"].min() > 1e-6
    Ad, Od = dev(A), dev(Om)
    g = R.decompose(ctx, Ad, Od, k, want_eta=True)
    assert g["status"] == 0 and g["status_I"] == 0
    assert np.array_equal(host(g["J"]).astype(np.int64), o["J"])
    assert np.array_equal(host(g["I"]).astype(np.int64), o["I"])
    Zg = host(g["Z"])
    kappa = np.linalg.cond(o["X"][:k][:, o["J"]])
    np.testing.assert_allclose(Zg, o["Z"], rtol=0, atol=1e-13 * kappa * max(1.0, np.abs(o["Z"]).max()))
    assert abs(g["eta"] - o["eta"]) <= 1e-6 * o["eta"]
    Ug = host(g["U"])
    np.testing.assert_allclose(Ug, o["U"], rtol=1e-7, atol=1e-7 * np.abs(o["U"]).max())
    ro = O.residuals(A, o["J"], Z=o["Z"], I=o["I"], U=o["U"])
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, g["J"], I=g["I"], U=g["U"])
    say("residuals gpu", rid, rcur, "oracle", ro["id"], ro["cur"])
    assert abs(rid - ro["id"]) <= 1e-9 * ro["id"]
    assert abs(rcur - ro["cur"]) <= 1e-9 * ro["cur"]


@pytest.mark.parametrize("m,n,k,l,seed", [(2048, 1800, 256, 272, 5), (1500, 1700, 200, 200, 6),
                                          (1300, 1100, 170, 180, 7), (2600, 2400, 400, 420, 8),
                                          (3000, 2600, 512, 544, 9)])
def test_large_k_f64_end_to_end(R, ctx, m, n, k, l, seed):
    """k above what one workgroup holds in registers (the triangular factors
    are split into 2 x 2 blocks up to 288, and a leading block of 128 is split
    off repeatedly above that: 400 and 512), k not a multiple of 32: J and I
    bit-exact, Z within its conditioning, U through the CUR residual (1e-9
    relative)."""
    say("large-k f64", m, n, k, l)
    A, Om = inputs.small_spectral_case(m, n, k, l, inputs.poly_spectrum(min(m, n), 1.0), seed)
    o = O.decompose(A, Om, k, gaps=True)
    assert o["gap_J"].min() > 1e-9 and o["gap_I"].min() > 1e-9
    Ad, Od = dev(A), dev(Om)
    g = R.decompose(ctx, Ad, Od, k, want_eta=True)
    assert g["status"] == 0 and g["status_I"] == 0
    assert np.array_equal(host(g["J"]).astype(np.int64), o["J"])
    assert np.array_equal(host(g["I"]).astype(np.int64), o["I"])
    Zg = host(g["Z"])
    kappa = np.linalg.cond(o["X"][:k][:, o["J"]])
    np.testing.assert_allclose(Zg, o["Z"], rtol=0, atol=1e-13 * kappa * max(1.0, np.abs(o["Z"]).max()))
    assert abs(g["eta"] - o["eta"]) <= 1e-6 * o["eta"]
    Ug = host(g["U"])
    np.testing.assert_allclose(Ug, o["U"], rtol=1e-6, atol=1e-6 * np.abs(o["U"]).max())
    ro = O.residuals(A, o["J"], Z=o["Z"], I=o["I"], U=o["U"], only=("id", "cur"))
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, g["J"], I=g["I"], U=g["U"])
    say("residuals gpu", rid, rcur, "oracle", ro["id"], ro["cur"])
    assert abs(rid - ro["id"]) <= 1e-9 * ro["id"]
    assert abs(rcur - ro["cur"]) <= 1e-9 * ro["cur"]


@pytest.mark.parametrize("m,n,k,l,seed", [(5, 7, 1, 1, 1), (33, 40, 1, 3, 2), (64, 31, 31, 31, 3),
                                          (9, 300, 9, 9, 4), (130, 97, 97, 100, 5)])
def test_degenerate_ranks_f64_end_to_end(R, ctx, m, n, k, l, seed):
    """The extreme ranks of Alg. 2: k = 1 (one sketch row, one pivot, 1 x 1
    triangular factors), k = n (every column is a pivot, Z a permutation of
    the identity) and k = m (the row LUPP of C takes every row), with m, n
    and l below one tile.  J and I bit-exact, Z and U within their
    conditioning; residuals to 1e-9 relative, or at round-off where the
    oracle's are (the selected columns or rows then span A)."""
    say("degenerate ranks f64", m, n, k, l)
    A, Om = inputs.small_spectral_case(m, n, k, l, np.linspace(1.0, 0.5, min(m, n)), 60 + seed)
    o = O.decompose(A, Om, k, gaps=True)
    assert o["gap_J"].min() > 1e-6 and o["gap_I"].min() > 1e-6
    Ad, Od = dev(A), dev(Om)
    g = R.decompose(ctx, Ad, Od, k)
    assert g["status"] == 0 and g["status_I"] == 0
    assert np.array_equal(host(g["J"]).astype(np.int64), o["J"])
    assert np.array_equal(host(g["I"]).astype(np.int64), o["I"])
    kappa = np.linalg.cond(o["X"][:k][:, o["J"]])
    np.testing.assert_allclose(host(g["Z"]), o["Z"], rtol=0,
                               atol=1e-13 * kappa * max(1.0, np.abs(o["Z"]).max()))
    np.testing.assert_allclose(host(g["U"]), o["U"], rtol=1e-7, atol=1e-7 * np.abs(o["U"]).max())
    ro = O.residuals(A, o["J"], Z=o["Z"], I=o["I"], U=o["U"], only=("id", "cur"))
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, g["J"], I=g["I"], U=g["U"])
    say("residuals gpu", rid, rcur, "oracle", ro["id"], ro["cur"])
    for rg, r in ((rid, ro["id"]), (rcur, ro["cur"])):
        if r > 1e-10:
            assert abs(rg - r) <= 1e-9 * r
        else:
            assert rg <= 1e-12


@pytest.mark.parametrize("m,n,k,seed", [(2600, 2200, 600, 11), (2100, 2300, 1024, 12)])
def test_id_beyond_512_f64(R, ctx, m, n, k, seed):
    """The interpolative decomposition at ranks above 512 (the triangular
    inverse behind Z is assembled from two half-order inverses): J bit-exact,
    Z within its conditioning, the ID residual to 1e-9 relative."""
    say("id beyond 512", m, n, k)
    A, Om = inputs.small_spectral_case(m, n, k, k, inputs.poly_spectrum(min(m, n), 1.0), seed)
    X = O.sketch(A, Om)
    f = O.lupp_colwise(X, k, gaps=True)
    assert f["gap"].min() > 1e-9
    Zo = O.id_coeffs(X, f["J"], k)
    Ad = dev(A)
    Xd = R.rpid_sketch(ctx, Ad, dev(Om))
    J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, Xd, k)
    assert st == 0 and keff == k
    assert np.array_equal(host(J).astype(np.int64), f["J"])
    Z, _ = R.rpid_id_coeffs(ctx, Xd, k, J, Lf, Uf, refine_steps=0)
    kappa = np.linalg.cond(X[:k][:, f["J"]])
    np.testing.assert_allclose(host(Z), Zo, rtol=0, atol=1e-13 * kappa * max(1.0, np.abs(Zo).max()))
    ro = O.residuals(A, f["J"], Z=Zo, only=("id",))["id"]
    rg = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, J, Z=Z)
    say("residual gpu", rg, "oracle", ro, "kappa", kappa)
    assert abs(rg - ro) <= 1e-9 * ro


@pytest.mark.parametrize("m,n,k,seed", [(300, 257, 16, 1), (1500, 900, 100, 2)])
def test_exact_recovery_gpu(R, ctx, m, n, k, seed):
    """rank(A) = k, l = k: the GPU's ID and CUR residuals are at round-off."""
    say("exact recovery", m, n, k)
    A, Om = inputs.small_spectral_case(m, n, k, k, np.linspace(1.0, 0.2, k), 40 + seed)
    Ad, Od = dev(A), dev(Om)
    g = R.decompose(ctx, Ad, Od, k)
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, g["J"], I=g["I"], U=g["U"])
    assert rid < 1e-12 and rcur < 1e-11, (rid, rcur)


@pytest.mark.parametrize("dt", ["float32", "bfloat16"])
def test_precision_modes_small(R, ctx, dt):
    """FP32 / BF16 storage on a polynomial-spectrum case: the GPU residuals
    stay within 1.05x of the FP64 oracle's on the same stored values."""
    m, n, k, l = 1200, 1000, 64, 80
    say("precision", dt, m, n, k, l)
    tdt = getattr(torch, dt)
    A, Om = inputs.small_spectral_case(m, n, k, l, inputs.poly_spectrum(min(m, n), 2.0), 77)
    Ad, Od = dev(A, tdt), dev(Om, tdt)
    a_s, o_s = host(Ad), host(Od)
    o = O.decompose(a_s, o_s, k)
    ro = O.residuals(a_s, o["J"], Z=o["Z"], I=o["I"], U=o["U"])
    g = R.decompose(ctx, Ad, Od, k)
    assert g["status"] == 0 and g["status_I"] == 0
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, g["J"], I=g["I"], U=g["U"])
    say("gpu", rid, rcur, "oracle", ro["id"], ro["cur"])
    assert rid <= 1.05 * ro["id"] and rcur <= 1.05 * ro["cur"]
    # the GPU's own residual evaluation agrees with the oracle's evaluation of
    # the GPU's decomposition
    rg = O.residuals(a_s, host(g["J"]).astype(np.int64), Z=host(g["Z"]),
                     I=host(g["I"]).astype(np.int64), U=host(g["U"]))
    assert abs(rid - rg["id"]) <= 1e-4 * rg["id"]
    assert abs(rcur - rg["cur"]) <= 1e-4 * rg["cur"]


@pytest.mark.parametrize("dt", ["float32", "bfloat16"])
@pytest.mark.parametrize("m,n,k,l", [(300, 257, 1, 1), (64, 31, 31, 31)])
def test_precision_modes_extreme_ranks(R, ctx, dt, m, n, k, l):
    """FP32 and BF16 storage at k = 1 (one sketch row; in BF16 the CUR's
    product W = Q_C^T A runs on two sketch rows) and at k = n.  k = 1: both
    residuals within 1.05x of the FP64 oracle's on the same stored values.
    k = n: Z is a permutation, so A - CZ vanishes exactly; the CUR residual
    stays at the precision of W's product (FP32: 2^-24; BF16: Q_C in two BF16
    terms, about 2^-16), bounded here by 1e-5 and 1e-3."""
    say("precision extreme ranks", dt, m, n, k, l)
    tdt = getattr(torch, dt)
    A, Om = inputs.small_spectral_case(m, n, k, l, np.linspace(1.0, 0.5, min(m, n)), 90 + k)
    Ad, Od = dev(A, tdt), dev(Om, tdt)
    g = R.decompose(ctx, Ad, Od, k)
    assert g["status"] == 0 and g["status_I"] == 0
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, g["J"], I=g["I"], U=g["U"])
    if k == n:
        say("gpu", rid, rcur)
        assert sorted(host(g["J"]).astype(np.int64).tolist()) == list(range(n))
        assert rid == 0.0
        assert rcur <= (1e-5 if dt == "float32" else 1e-3)
    else:
        a_s, o_s = host(Ad), host(Od)
        o = O.decompose(a_s, o_s, k)
        ro = O.residuals(a_s, o["J"], Z=o["Z"], I=o["I"], U=o["U"], only=("id", "cur"))
        say("gpu", rid, rcur, "oracle", ro["id"], ro["cur"])
        assert rid <= 1.05 * ro["id"] and rcur <= 1.05 * ro["cur"]


def test_argument_validation(R, ctx):
    """Invalid arguments return -position; nothing is launched."""
    say("validation")
    X = dev(np.ones((4, 10)))
    with pytest.raises(R.RpidError) as e:
        R.rpid_select_columns(ctx, X, 5)  # k > l
    assert e.value.status == -7
    A = dev(np.ones((10, 12)))
    Om = dev(np.ones((3, 10)))
    with pytest.raises(R.RpidError) as e:
        R.rpid_sketch(ctx, A, dev(np.ones((3, 10)), torch.float32))  # mixed types
    assert e.value.status == -103
