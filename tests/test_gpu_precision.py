"""GPU tests of the precision forms: the FP8 (E4M3) sketch against the FP64
oracle of the same quantisation, the tall non-negative FP8 workload end to
end (CUR), the LUPP at the tall workload's full panel size, and the BF16
path at k = 512 (the Cholesky-QR and inverse kernels beyond registers)."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.rpid_oracle as O  # noqa: E402
from paper_2104_05877_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print("[precision]", *a, flush=True)


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


def fp8_bound(A, Om):
    """FP32 accumulation bound for the E4M3 sketch: 2 m u32 (|Om_q| |A_q|)
    in the unscaled units (the products of E4M3 values are exact in FP32)."""
    ea = np.array([O.fp8_scale_exp(np.abs(A[:, j]).max()) for j in range(A.shape[1])])
    eo = O.fp8_scale_exp(np.abs(Om).max())
    Aq = np.abs(O.e4m3_round(A * np.ldexp(1.0, ea)[None, :]))
    Oq = np.abs(O.e4m3_round(Om * np.ldexp(1.0, eo)))
    m = A.shape[0]
    return 2 * m * 2.0**-24 * (Oq @ Aq) * np.ldexp(1.0, -(eo + ea))[None, :]


@pytest.mark.parametrize("m,n,l,seed", [(1000, 800, 50, 1), (4096, 515, 400, 2), (777, 33, 17, 3),
                                        (65536, 96, 400, 4)])
def test_sketch_fp8_parity(R, ctx, m, n, l, seed):
    """E4M3 sketch with per-column and global power-of-two scales vs the
    oracle's exact product of the same quantised values (ragged m is padded
    with zero codes; l = 400 spans two row chunks)."""
    say("sketch fp8", m, n, l)
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((m, n)) * 10.0 ** rng.uniform(-3, 3, n)[None, :]).astype(np.float32)
    Om = rng.standard_normal((l, m)).astype(np.float32)
    Ad = inputs.torch_colmajor(A, torch.float32, "cuda")
    Od = inputs.torch_colmajor(Om, torch.float32, "cuda")
    X = host(R.rpid_sketch_fp8(ctx, Ad, Od))
    ref = O.sketch_fp8(A.astype(np.float64), Om.astype(np.float64))
    bound = fp8_bound(A.astype(np.float64), Om.astype(np.float64))
    assert np.all(np.abs(X - ref) <= bound + 1e-300)


def test_sketch_fp8_tall_full_size_sampled(R, ctx):
    """The tall workload at full size (65536 x 4096, l = 400): sampled
    columns of X against the oracle, which needs only those columns of A."""
    m, n, r, l = 65536, 4096, 384, 400
    say("sketch fp8 full size", m, n, l)
    Ad = inputs.torch_nonneg_lowrank(m, n, r, 1e-3, 5, "cuda")
    Od = inputs.torch_gaussian(l, m, 6, "cuda", dtype=torch.float32)
    X = R.rpid_sketch_fp8(ctx, Ad, Od)
    cols = np.array([0, 1, 17, 1000, 2047, 2048, 3001, 4095])
    A = Ad[:, torch.tensor(cols, device="cuda")].double().cpu().numpy()
    Om = Od.double().cpu().numpy()
    ref = O.sketch_fp8(A, Om)
    Xs = host(X)[:, cols]
    assert np.all(np.abs(Xs - ref) <= fp8_bound(A, Om) + 1e-300)


def test_lupp_tall_panel_invariants(R, ctx):
    """FP32 LUPP of a 384 x 65536 panel (256 workgroups of 768 threads, two
    threads per column, one workgroup per CU): pivots distinct, |L'| <= 1
    with unit pivots, and X^T(:, 0:k) = L' U' (the row order of L' is the
    original one) to FP32 accuracy."""
    l, n, k = 384, 65536, 384
    say("lupp tall panel", l, n, k)
    X = inputs.torch_gaussian(l, n, 21, "cuda", dtype=torch.float32)
    J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, X, k)
    assert st == 0 and keff == k
    Jh = J.cpu().numpy()
    assert len(np.unique(Jh)) == k
    L_ = host(Lf)
    assert np.abs(L_).max() <= 1.0 + 1e-6
    assert np.all(L_[Jh, np.arange(k)] == 1.0)
    U_ = host(Uf)
    Xt = host(X)[:k].T
    err = np.abs(Xt - L_ @ U_).max() / np.abs(Xt).max()
    say("reconstruction", err)
    assert err < 1e-3


def test_tall_fp8_cur_end_to_end(R, ctx):
    """A scaled-down tall non-negative workload: FP8 sketch, FP32 LUPP, CUR
    from the FP32 values.  The CUR residual stays within 1.05x of the oracle
    running the same FP8 quantisation in FP64, or within the spread of the
    oracle over five sketches (the residual sits at the noise floor)."""
    m, n, r, k, l = 8192, 1024, 64, 64, 72
    say("tall fp8 cur", m, n, k, l)
    Ad = inputs.torch_nonneg_lowrank(m, n, r, 1e-3, 7, "cuda")
    A = Ad.double().cpu().numpy()
    res_o = []
    for s in range(5):
        Od = inputs.torch_gaussian(l, m, 30 + s, "cuda", dtype=torch.float32)
        Om = Od.double().cpu().numpy()
        X = O.sketch_fp8(A, Om)
        J = O.lupp_colwise(X, k)["J"]
        I = O.lupp_rowwise(A[:, J], k)["J"]
        U = O.cur_u(A, J, I)
        res_o.append(O.residuals(A, J, I=I, U=U, only=("cur",))["cur"])
        if s == 0:
            Xg = R.rpid_sketch_fp8(ctx, Ad, Od)
            Jg, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, Xg, k)
            assert st == 0
            Ig, Ug, keff_i, st_i = R.rpid_cur(ctx, Ad, k, Jg)
            assert st_i == 0
            rg = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, Jg, I=Ig, U=Ug)
    say("gpu", rg, "oracle", res_o)
    assert rg <= 1.05 * res_o[0] or rg <= max(res_o)


def test_bf16_k512_end_to_end(R, ctx):
    """BF16 storage at k = 512, l = 544 (LUPP with 512 columns, Cholesky-QR and
    triangular inverses beyond the register-resident size): ID and CUR
    residuals within 1.05x of the FP64 oracle on the same stored values."""
    m, n, k, l = 4096, 3000, 512, 544
    say("bf16 k512", m, n, k, l)
    A64 = inputs.torch_lowrank_noise(m, n, k, 1e-4, 9, "cuda")
    Ab = A64.T.contiguous().bfloat16().T
    Ob = inputs.torch_gaussian(l, m, 10, "cuda").T.contiguous().bfloat16().T
    g = R.decompose(ctx, Ab, Ob, k)
    assert g["status"] == 0 and g["status_I"] == 0
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ab, k, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ab, k, g["J"], I=g["I"], U=g["U"])
    A = host(Ab)
    o = O.decompose(A, host(Ob), k)
    ro = O.residuals(A, o["J"], Z=o["Z"], I=o["I"], U=o["U"], only=("id", "cur"))
    say("gpu", rid, rcur, "oracle", ro["id"], ro["cur"])
    assert rid <= 1.05 * ro["id"] and rcur <= 1.05 * ro["cur"]


@pytest.mark.parametrize("m,n,k,seed", [(1000, 700, 64, 1), (2048, 1536, 128, 2), (777, 300, 192, 3),
                                        (640, 513, 50, 4)])
def test_bf16_residual_against_oracle(R, ctx, m, n, k, seed):
    """BF16-storage residuals (BF16 MFMA with FP32 accumulation over the
    three-term BF16 split of the FP64 factor) against the FP64 oracle's
    explicit differences on the same stored values: |r_gpu - r_oracle|
    ||A|| <= gamma || |P| |Q| ||_F with gamma = (3 k + 3) 2^-24 (FP32
    accumulation over 3 k terms plus the split's remainder).  k = 64, 128,
    192 take the streaming kernel (ragged 128 x 128 tiles at these m, n);
    k = 50 the general one."""
    say("bf16 residual", m, n, k)
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((m, n)) * 10.0 ** rng.uniform(-1, 1, n)[None, :])
    Ad = inputs.torch_colmajor(A, torch.bfloat16, "cuda")
    a_s = host(Ad)
    J = np.sort(rng.choice(n, k, replace=False)).astype(np.int64)
    I = np.sort(rng.choice(m, k, replace=False)).astype(np.int64)
    C = a_s[:, J]
    # Z and U that leave a moderate residual (a least-squares fit plus noise)
    Z = np.linalg.lstsq(C, a_s, rcond=None)[0] + 1e-3 * rng.standard_normal((k, n))
    Rr = a_s[I, :]
    U = np.linalg.pinv(C) @ a_s @ np.linalg.pinv(Rr) + 1e-3 * rng.standard_normal((k, k))
    Jd = torch.tensor(J, device="cuda")
    Id = torch.tensor(I, device="cuda")
    gamma = (3 * k + 3) * 2.0**-24
    na = np.linalg.norm(a_s)
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, Jd, Z=torch.tensor(Z.T.copy(), device="cuda").T)
    ro = O.residuals(a_s, J, Z=Z, only=("id",))["id"]
    bound = gamma * np.linalg.norm(np.abs(C) @ np.abs(Z)) / na
    say("id", rid, ro, bound)
    assert abs(rid - ro) <= bound + 1e-12
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, Jd, I=Id, U=torch.tensor(U.T.copy(), device="cuda").T)
    ro = O.residuals(a_s, J, I=I, U=U, only=("cur",))["cur"]
    bound = gamma * np.linalg.norm(np.abs(C @ U) @ np.abs(Rr)) / na
    say("cur", rcur, ro, bound)
    assert abs(rcur - ro) <= bound + 1e-12



@pytest.mark.parametrize("m,l", [(302, 302), (70003, 300)])
def test_fp8_codes_ties_and_subnormals_exact(R, ctx, m, l):
    """The E4M3 codes themselves, exactly: Omega's rows are unit vectors
    (scale 2^8, codes 256 exactly), so each row of X is one quantised row of A,
    unscaled exactly.  Every column holds 448 (so its scale is 1), exact E4M3
    values, midpoints of consecutive codes over the whole range including the
    subnormals (ties: the even code must win) and arbitrary values.  m = 302
    (all rows selected) leaves a ragged tail of two rows after the last group
    of four; m = 70003 takes the two-pass quantisation of columns longer than
    65536 rows (rows selected at random, plus the last ten)."""
    n = 40
    rng = np.random.default_rng(11)
    table = O.e4m3_values()
    k = rng.integers(0, table.size - 1, size=(m, n))
    mids = (table[k] + table[k + 1]) / 2.0
    even = np.where(k % 2 == 0, k, k + 1)
    kind = rng.integers(0, 4, size=(m, n))  # 0, 1: midpoint, 2: exact value, 3: arbitrary
    A = np.where(kind <= 1, mids, np.where(kind == 2, table[k], rng.uniform(0.0, 448.0, (m, n))))
    A = A * np.where(rng.random((m, n)) < 0.5, -1.0, 1.0)
    A[0, :] = 448.0
    A = A.astype(np.float32).astype(np.float64)
    if l == m:
        rows = np.arange(m)
    else:
        rows = np.concatenate([np.sort(rng.choice(m - 10, l - 10, replace=False)), np.arange(m - 10, m)])
    Om = np.zeros((l, m))
    Om[np.arange(l), rows] = 1.0
    say("fp8 codes", m, n, l)
    X = host(R.rpid_sketch_fp8(ctx, inputs.torch_colmajor(A, torch.float32, "cuda"),
                               inputs.torch_colmajor(Om, torch.float32, "cuda")))
    expect = np.sign(A) * np.where(kind <= 1, table[even], np.where(kind == 2, table[k], np.nan))
    sel = kind <= 2
    sel[0, :] = False
    assert np.array_equal(X[sel[rows]], expect[rows][sel[rows]])
    assert np.array_equal(X, O.sketch_fp8(A, Om))


@pytest.mark.parametrize("m,n,l", [(4096, 48, 300), (65536, 8, 300)])
def test_fp8_codes_scaled_columns_exact(R, ctx, m, n, l):
    """The E4M3 codes exactly at row counts that are whole multiples of 2048
    (16-byte loads, the column kept as sign, exponent, top 4 mantissa bits
    and a sticky bit), over per-column scales from 2^30 down to 2^-150:
    column j is a column of midpoints of consecutive codes (ties), exact
    codes and arbitrary values, times 2^-s_j, with 448 2^-s_j in row 0 (so
    its scale exponent is s_j) and FP32 subnormals in rows 1..6 (scaled
    down with the column past s_j = 116, so that row 0 stays largest).  Scale
    exponents above 116 take the exact re-read of the column, and the
    subnormals must land on the same codes as in the oracle's FP64
    arithmetic at every scale."""
    rng = np.random.default_rng(17)
    table = O.e4m3_values()
    k = rng.integers(0, table.size - 1, size=(m, n))
    mids = (table[k] + table[k + 1]) / 2.0
    kind = rng.integers(0, 3, size=(m, n))  # 0: midpoint, 1: exact value, 2: arbitrary
    base = np.where(kind == 0, mids, np.where(kind == 1, table[k], rng.uniform(0.0, 448.0, (m, n))))
    base = base * np.where(rng.random((m, n)) < 0.5, -1.0, 1.0)
    base[0, :] = 448.0
    s = np.round(np.linspace(-30, 150, n)).astype(int)
    if n >= 8:
        s[1:4] = [116, 117, 120]
    A = base * np.ldexp(1.0, -s)[None, :]
    tiny = np.array([2.0**-127, -(2.0**-130), 3 * 2.0**-149, 2.0**-149, -1.5 * 2.0**-127, 2.0**-140])
    A[1:7, :] = tiny[:, None] * np.ldexp(1.0, -np.maximum(s - 116, 0))[None, :]
    A = A.astype(np.float32).astype(np.float64)
    assert all(O.fp8_scale_exp(np.abs(A[:, j]).max()) == s[j] for j in range(n))
    rows = np.concatenate([np.arange(7), np.sort(rng.choice(np.arange(7, m), l - 7, replace=False))])
    Om = np.zeros((l, m))
    Om[np.arange(l), rows] = 1.0
    say("fp8 codes scaled", m, n, l)
    X = host(R.rpid_sketch_fp8(ctx, inputs.torch_colmajor(A, torch.float32, "cuda"),
                               inputs.torch_colmajor(Om, torch.float32, "cuda")))
    assert np.array_equal(X, O.sketch_fp8(A, Om))


def test_fp8_contiguous_and_strided_paths_agree(R, ctx):
    """The FP8 sketch through its contiguous kernels (16-byte loads of whole
    2048-row groups of A, the flat maximum of Omega) and through its general
    ones (A and Omega as strided views, leading dimensions rows + 1): X
    bitwise equal, finite input or not.  A non-finite entry of A gives a NaN
    column of X (that column unscaled), a NaN in Omega a NaN row (Omega
    unscaled); the other columns keep the finite case's values bit for bit."""
    m, n, l = 4096, 40, 48
    say("fp8 paths", m, n, l)
    rng = np.random.default_rng(23)
    A0 = (rng.standard_normal((m, n)) * 10.0 ** rng.uniform(-3, 3, n)[None, :]).astype(np.float32)
    Om0 = rng.standard_normal((l, m)).astype(np.float32)

    def strided(M):
        r, c = M.shape
        buf = torch.zeros((c, r + 1), dtype=torch.float32, device="cuda")
        buf[:, :r] = torch.from_numpy(np.ascontiguousarray(M.T)).cuda()
        return buf[:, :r].T

    X_fin = None
    for case in ("finite", "A_nonfinite", "Om_nan"):
        A, Om = A0.copy(), Om0.copy()
        if case == "A_nonfinite":
            A[5, 3], A[7, 9] = np.nan, np.inf
        if case == "Om_nan":
            Om[2, 100] = np.nan
        Ac = inputs.torch_colmajor(A, torch.float32, "cuda")
        Oc = inputs.torch_colmajor(Om, torch.float32, "cuda")
        As, Os = strided(A), strided(Om)
        assert As.stride() == (1, m + 1) and Os.stride() == (1, l + 1)
        X1 = host(R.rpid_sketch_fp8(ctx, Ac, Oc))
        X2 = host(R.rpid_sketch_fp8(ctx, As, Os))
        assert np.array_equal(X1, X2, equal_nan=True), case
        if case == "finite":
            assert np.all(np.isfinite(X1))
            X_fin = X1
        elif case == "A_nonfinite":
            bad = np.zeros(n, dtype=bool)
            bad[[3, 9]] = True
            assert np.all(np.isnan(X1[:, bad]))
            assert np.array_equal(X1[:, ~bad], X_fin[:, ~bad])
        else:
            assert np.all(np.isnan(X1[2, :]))
            assert np.all(np.isfinite(np.delete(X1, 2, axis=0)))


def test_lupp_grid_above_one_workgroup_per_cu_refused(R, ctx):
    """A panel that would need more workgroups than compute units (FP64, k =
    384, 65536 rows: 128 rows per workgroup at most) is refused on the host
    with RPID_ERR_UNSUPPORTED; nothing is launched."""
    say("lupp refused grid", 384, 65536)
    X = inputs.torch_gaussian(384, 65536, 22, "cuda")
    with pytest.raises(R.RpidError) as e:
        R.rpid_select_columns(ctx, X, 384)
    assert e.value.status == -103


@pytest.mark.skip(reason="grids of more than one workgroup per compute unit are refused: one such "
                         "launch (two workgroups per CU, FP32 384 x 65536 panel) once ran into the "
                         "exchange's spin limit and the cause has not been shown")
def test_lupp_two_workgroups_per_cu():
    """Kept as a record of the refused configuration (see the reason)."""
