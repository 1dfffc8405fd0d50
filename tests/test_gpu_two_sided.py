"""GPU tests of the streaming skeleton selection of Alg. 3 against the FP64
oracle: the two-sided sketch X = Gamma A, Y = A Omega^T (returned as Y^T),
row pivoting on Y, the row ID estimated from Y, and the cheap CUR core
S^{-1} = A(I, J)^{-1}."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.rpid_oracle as O  # noqa: E402
from paper_2104_05877_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print("[two-sided]", *a, flush=True)


@pytest.fixture(scope="module")
def R():
    from paper_2104_05877_amd import rpid

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return rpid


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


def host(t):
    return t.detach().double().cpu().numpy()


def dev(a, dt, pad=0):
    """Column-major device copy; pad > 0 gives lda = rows + pad."""
    if pad == 0:
        return inputs.torch_colmajor(a, dt, "cuda")
    big = np.zeros((a.shape[0] + pad, a.shape[1]))
    big[: a.shape[0]] = a
    return inputs.torch_colmajor(big, dt, "cuda")[: a.shape[0]]


U_ROUND = {"float64": 2.0**-53, "float32": 2.0**-24, "bfloat16": 2.0**-24}

# (m, n, l, pad, seed).  BF16 reads A in place when n % 64 == 0 and m % 8 ==
# 0 (then m = 8200, n = 16384 takes three row blocks of 4096, 4096 and 8
# rows); the other shapes take the transposed-copy path.
CASES = [
    (1000, 800, 60, 0, 1),
    (1000, 512, 272, 0, 2),
    (1024, 2048, 64, 24, 3),
    (777, 640, 40, 0, 4),
]
# every storage type on the small shapes; the multi-block in-place read
# (m = 8200, n = 16384) exists only for BF16 storage
SKETCH_CASES = [(dt,) + c for c in CASES for dt in ("float64", "float32", "bfloat16")] + [
    ("bfloat16", 8200, 16384, 64, 0, 5)]


@pytest.mark.parametrize("dt,m,n,l,pad,seed", SKETCH_CASES)
def test_two_sided_sketch_against_oracle(R, ctx, m, n, l, pad, seed, dt):
    """|X - Gamma A| <= 2 (m + 2) u |Gamma| |A| and |Y - A Omega^T| <=
    2 (n + 2) u |A| |Omega|^T elementwise, on the stored values."""
    say("sketch", dt, m, n, l, "pad", pad)
    tdt = getattr(torch, dt)
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * 10.0 ** rng.uniform(-1, 1, n)[None, :]
    G = rng.standard_normal((l, m))
    Om = rng.standard_normal((l, n))
    Ad, Gd, Od = dev(A, tdt, pad), dev(G, tdt), dev(Om, tdt)
    a_s, g_s, o_s = host(Ad), host(Gd), host(Od)
    X, Yt = R.rpid_sketch_two_sided(ctx, Ad, Gd, Od)
    assert X.shape == (l, n) and Yt.shape == (l, m)
    Xo, Yo = O.sketch_two_sided(a_s, g_s, o_s)
    u = U_ROUND[dt]
    bx = 2 * (m + 2) * u * (np.abs(g_s) @ np.abs(a_s))
    by = 2 * (n + 2) * u * (np.abs(a_s) @ np.abs(o_s).T)
    ex = np.abs(host(X) - Xo)
    ey = np.abs(host(Yt).T - Yo)
    say("max err/bound X", float((ex / bx).max()), "Y", float((ey / by).max()))
    assert np.all(ex <= bx) and np.all(ey <= by)


def _two_sided_fp64_case(R, ctx, A, G, Om, k):
    Ad = dev(A, torch.float64)
    X, Yt = R.rpid_sketch_two_sided(ctx, Ad, dev(G, torch.float64), dev(Om, torch.float64))
    o = O.decompose_two_sided(A, G, Om, k, gaps=True)
    assert o["gap_J"].min() > 1e-9 and o["gap_I"].min() > 1e-9
    J, Lf, Uf, _, keff, st = R.rpid_select_columns(ctx, X, k)
    I, Li, Ui, _, keff_i, st_i = R.rpid_select_columns(ctx, Yt, k)
    assert st == 0 and st_i == 0
    assert np.array_equal(J.cpu().numpy(), o["J"]) and np.array_equal(I.cpu().numpy(), o["I"])
    Zy, _ = R.rpid_id_coeffs(ctx, Yt, k, I, Li, Ui)
    W = host(Zy).T
    np.testing.assert_allclose(W, o["W"], rtol=0, atol=1e-8 * np.abs(o["W"]).max())
    Us, s = R.rpid_cur_sketch(ctx, Ad, k, J, I)
    assert s == 0
    kappa = np.linalg.cond(A[np.ix_(o["I"], o["J"])])
    np.testing.assert_allclose(host(Us), o["U_sketch"], rtol=0,
                               atol=1e-14 * kappa * np.abs(o["U_sketch"]).max())
    r_row = R.rpid_residual(ctx, R.RESIDUAL_ROW_ID, Ad, k, None, Z=Zy, I=I)
    r_cur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, J, I=I, U=Us)
    ro = O.residuals(A, o["J"], I=o["I"], U=o["U_sketch"], W=o["W"], only=("rowid", "cur"))
    say("row id", r_row, ro["rowid"], "cheap cur", r_cur, ro["cur"])
    for rg, r in ((r_row, ro["rowid"]), (r_cur, ro["cur"])):
        if r > 1e-10:
            assert abs(rg - r) <= 1e-9 * r
        else:  # the selected rows or columns span A: round-off
            assert rg <= 1e-12


def test_two_sided_fp64_decomposition(R, ctx):
    """FP64 end to end: J from X and I from Y equal the oracle's (no near-ties
    on this input), the row ID from Y (rpid_id_coeffs on Y^T) and the cheap
    core S^{-1} match the oracle's within their conditioning, and the row ID
    and cheap CUR residuals match to 1e-9 relative."""
    m, n, k, l = 1200, 1000, 40, 48
    A, _ = inputs.small_spectral_case(m, n, k, l, inputs.poly_spectrum(min(m, n), 2.0), 11)
    rng = np.random.default_rng(12)
    G, Om = rng.standard_normal((l, m)), rng.standard_normal((l, n))
    _two_sided_fp64_case(R, ctx, A, G, Om, k)


@pytest.mark.parametrize("m,n,k,l,seed", [(7, 5, 1, 1, 1), (40, 33, 33, 33, 2), (30, 50, 30, 30, 3)])
def test_two_sided_fp64_extreme_ranks(R, ctx, m, n, k, l, seed):
    """Alg. 3 at k = 1 with one sketch row on each side, at k = n (every
    column a pivot) and at k = m (every row a pivot): the same checks, with
    the residuals at round-off where the pivots span A."""
    say("two-sided extreme ranks", m, n, k, l)
    A, _ = inputs.small_spectral_case(m, n, k, l, np.linspace(1.0, 0.5, min(m, n)), 70 + seed)
    rng = np.random.default_rng(80 + seed)
    G, Om = rng.standard_normal((l, m)), rng.standard_normal((l, n))
    _two_sided_fp64_case(R, ctx, A, G, Om, k)


@pytest.mark.parametrize("m,n,k,l", [(2048, 1536, 64, 80), (4096, 4096, 128, 144)])
def test_two_sided_bf16_decomposition(R, ctx, m, n, k, l):
    """BF16 storage (single-pass sketch): the row ID, cheap CUR and column ID
    residuals built on the GPU sketches stay within 1.05x of the FP64
    oracle's on the same stored values."""
    say("bf16 decomposition", m, n, k, l)
    A, _ = inputs.small_spectral_case(m, n, k, l, inputs.poly_spectrum(min(m, n), 2.0), 13)
    rng = np.random.default_rng(14)
    G, Om = rng.standard_normal((l, m)), rng.standard_normal((l, n))
    Ad, Gd, Od = dev(A, torch.bfloat16), dev(G, torch.bfloat16), dev(Om, torch.bfloat16)
    a_s, g_s, o_s = host(Ad), host(Gd), host(Od)
    X, Yt = R.rpid_sketch_two_sided(ctx, Ad, Gd, Od)
    J, Lf, Uf, _, _, st = R.rpid_select_columns(ctx, X, k)
    I, Li, Ui, _, _, st_i = R.rpid_select_columns(ctx, Yt, k)
    assert st == 0 and st_i == 0
    Z, _ = R.rpid_id_coeffs(ctx, X, k, J, Lf, Uf, refine_steps=1)
    Zy, _ = R.rpid_id_coeffs(ctx, Yt, k, I, Li, Ui, refine_steps=1)
    Us, s = R.rpid_cur_sketch(ctx, Ad, k, J, I)
    assert s == 0
    r_id = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, J, Z=Z)
    r_row = R.rpid_residual(ctx, R.RESIDUAL_ROW_ID, Ad, k, None, Z=Zy, I=I)
    r_cur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, J, I=I, U=Us)
    o = O.decompose_two_sided(a_s, g_s, o_s, k)
    ro = O.residuals(a_s, o["J"], Z=o["Z"], I=o["I"], U=o["U_sketch"], W=o["W"], only=("id", "rowid", "cur"))
    say("id", r_id, ro["id"], "row id", r_row, ro["rowid"], "cheap cur", r_cur, ro["cur"])
    assert r_id <= 1.05 * ro["id"]
    assert r_row <= 1.05 * ro["rowid"]
    assert r_cur <= 1.05 * ro["cur"]


def test_cur_sketch_zero_pivot(R, ctx):
    """S = A(I, J) with a zero column (the third) is singular: the LU of S
    meets an exactly zero pivot at its third step, so the status is 3 (the
    1-based step), with no exception."""
    rng = np.random.default_rng(15)
    A = rng.standard_normal((64, 48))
    A[[0, 5, 9, 30], 7] = 0.0
    Ad = dev(A, torch.float64)
    J = torch.tensor([3, 10, 7, 20], dtype=torch.int64, device="cuda")
    I = torch.tensor([0, 5, 9, 30], dtype=torch.int64, device="cuda")
    U, s = R.rpid_cur_sketch(ctx, Ad, 4, J, I)
    assert s == 3


def test_two_sided_argument_errors(R, ctx):
    A = dev(np.zeros((64, 32)), torch.float64)
    G = dev(np.zeros((8, 64)), torch.float64)
    Om = dev(np.zeros((8, 32)), torch.float64)
    with pytest.raises(ValueError):
        R.rpid_sketch_two_sided(ctx, A, Om, Om)
    with pytest.raises(ValueError):
        R.rpid_sketch_two_sided(ctx, A, G.float(), Om)
    big = dev(np.zeros((1100, 64)), torch.float64)
    with pytest.raises(R.RpidError) as e:
        R.rpid_sketch_two_sided(ctx, A, big, dev(np.zeros((1100, 32)), torch.float64))
    assert e.value.status == -11
