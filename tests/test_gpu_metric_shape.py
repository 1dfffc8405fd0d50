"""The path at the sizes of the benchmark and of the precision forms, through
the C-ABI, against the CPU oracle on the same stored values.

* 8192 x 8192, s_i = i^-2, k = 256, l = 272 (the benchmark workload), in the
  FP64, FP32 and BF16 modes;
* 16384 x 16384 stored BF16 (rank-512 Gaussian factors + 1e-4 noise),
  k = 512, l = 544;
* 65536 x 4096 non-negative (rank 384 + uniform[0, 1e-3] noise) with the FP8
  sketch, k = 384, l = 400, CUR.

Gates: in FP64 mode J and I equal the oracle's (with the near-tie audit of a
first differing step, should there be one) and every output agrees within
its conditioning; in every mode the LUPPs are bit-exact (pivots, multipliers
and U') against the oracle's fixed-arithmetic LUPP (correctly rounded
division, fused Schur update) run in the kernel's precision on the kernel's
own input, and the residuals stay within 1.05x of the FP64 oracle's on the
same stored values.  Each case prints the error against the FP64 oracle of
X, Z and U.
"""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.rpid_oracle as O  # noqa: E402
from paper_2104_05877_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

M = N = 8192
K, L = 256, 272
U64 = 2.0**-53
U32 = 2.0**-24


def say(*a):
    print("[metric-shape]", *a, flush=True)


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


def host(t):
    return t.detach().double().cpu().numpy()


def hint(t):
    return t.detach().cpu().numpy().astype(np.int64)


@pytest.fixture(scope="module")
def poly8192(R):
    say("generating poly8192 (seed 1)")
    a32, om32 = inputs.torch_poly8192(1, "cuda")
    torch.cuda.synchronize()
    return a32, om32


@pytest.fixture(scope="module")
def oracle_fp32_values(poly8192):
    """The FP64 oracle on the FP32-stored values (the inputs of the FP64 and
    FP32 modes): the numpy oracle with per-step pivot gaps."""
    a32, om32 = poly8192
    A, Om = host(a32), host(om32)
    say("oracle on the FP32 values")
    o = O.decompose(A, Om, K, gaps=True)
    o["res"] = O.residuals(A, o["J"], Z=o["Z"], I=o["I"], U=o["U"], only=("id", "cur"))
    return A, Om, o


def near_tie_audit(Jg, Jo, gaps, X, t_unit):
    """Length of the common pivot prefix, and whether a first difference is
    explained by a near tie: the oracle's relative gap at that step below
    64 m u (the rounding of the Schur complements)."""
    same = Jg == Jo
    p = int(np.argmin(same)) if not same.all() else len(Jo)
    explained = p == len(Jo) or gaps[p] < 64 * X.shape[1] * t_unit
    return p, explained


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_poly8192_f64_bit_exact(R, ctx, poly8192, oracle_fp32_values):
    """FP64 mode at the benchmark size: J and I equal the oracle's; the LUPP
    factors equal the fixed-arithmetic oracle's bit for bit; X, Z, U and both
    residuals agree within their conditioning."""
    A, Om, o = oracle_fp32_values
    a32, om32 = poly8192
    Ad = a32.T.contiguous().double().T
    Od = om32.T.contiguous().double().T
    say("f64 mode", M, N, K, L)
    g = R.decompose(ctx, Ad, Od, K)
    assert g["status"] == 0 and g["status_I"] == 0
    Xg = host(g["X"])
    # X: any summation order stays within 8 sqrt(m) u |Omega| |A|
    bound = 8 * np.sqrt(M) * U64 * (np.abs(Om) @ np.abs(A))
    assert np.all(np.abs(Xg - o["X"]) <= bound)
    # the column LUPP on the kernel's own X, bit for bit
    f = O.lupp_colwise_fma(Xg, K, np.float64)
    assert np.array_equal(hint(g["J"]), f["J"])
    assert np.array_equal(host(g["Lf"]), f["L"])
    assert np.array_equal(host(g["Uf"]), f["U"])
    # pivots against the numpy oracle on its own sketch
    Jg, Ig = hint(g["J"]), hint(g["I"])
    p, ok = near_tie_audit(Jg, o["J"], o["gap_J"], o["X"], U64)
    say("J common prefix", p, "of", K)
    assert ok, ("J differs without a near tie", p, o["gap_J"][p])
    assert np.array_equal(Jg, o["J"])
    q, ok = near_tie_audit(Ig, o["I"], o["gap_I"], A, U64)
    say("I common prefix", q, "of", K)
    assert np.array_equal(Ig, o["I"])
    # the row LUPP on C, bit for bit
    fr = O.lupp_colwise_fma(A[:, Jg].T, K, np.float64)
    assert np.array_equal(Ig, fr["J"])
    Zg, Ug = host(g["Z"]), host(g["U"])
    kappa = np.linalg.cond(o["X"][:K][:, o["J"]])
    ez, eu = rel(Zg, o["Z"]), rel(Ug, o["U"])
    say("kappa(X_1)", kappa, "rel err X", rel(Xg, o["X"]), "Z", ez, "U", eu)
    assert ez <= 1e-13 * kappa
    assert eu <= 1e-7
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, K, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, K, g["J"], I=g["I"], U=g["U"])
    say("residuals gpu", rid, rcur, "oracle", o["res"]["id"], o["res"]["cur"])
    assert abs(rid - o["res"]["id"]) <= 1e-9 * o["res"]["id"]
    assert abs(rcur - o["res"]["cur"]) <= 1e-9 * o["res"]["cur"]


def _low_precision_mode(R, ctx, Ad, Od, A, Om, o, name):
    """FP32 / BF16 storage: sketch within the FP32 accumulation bound, the FP32
    LUPPs bit-exact against the fixed-arithmetic oracle in float32 on the
    kernel's own inputs, residuals within 1.05x of the FP64 oracle's, and the
    errors of X, Z, U against it."""
    g = R.decompose(ctx, Ad, Od, K)
    assert g["status"] == 0 and g["status_I"] == 0
    Xg = host(g["X"])
    err_x = np.abs(Xg - o["X"])
    assert np.all(err_x <= 2 * M * U32 * (np.abs(Om) @ np.abs(A)))
    f = O.lupp_colwise_fma(Xg, K, np.float32)
    Jg, Ig = hint(g["J"]), hint(g["I"])
    assert np.array_equal(Jg, f["J"])
    assert np.array_equal(host(g["Lf"]), f["L"].astype(np.float64))
    assert np.array_equal(host(g["Uf"]), f["U"].astype(np.float64))
    fr = O.lupp_colwise_fma(A[:, Jg].T, K, np.float32)
    assert np.array_equal(Ig, fr["J"])
    p, _ = near_tie_audit(Jg, o["J"], o["gap_J"], o["X"], U32)
    overlap = len(np.intersect1d(Jg, o["J"])) / K
    out = dict(J_prefix=p, J_overlap=overlap, X_rel_err=rel(Xg, o["X"]))
    if p == K:
        # Z of the FP32 sketch after one FP64 refinement step against the
        # oracle's Z: first-order perturbation of Z = X_1^{-1} X_k by the
        # sketch's error E: |dZ| <= ||X_1^{-1}|| (||E_k|| + ||E_1|| ||Z||)
        Zg = host(g["Z"])
        Xk = o["X"][:K]
        E = Xg[:K] - Xk
        inv_n = 1.0 / np.linalg.svd(Xk[:, Jg], compute_uv=False)[-1]
        zb = inv_n * (np.linalg.norm(E, 2) + np.linalg.norm(E[:, Jg], 2) * np.linalg.norm(o["Z"], 2))
        dz = np.linalg.norm(Zg - o["Z"], 2)
        out.update(Z_rel_err=rel(Zg, o["Z"]), Z_err_2norm=dz, Z_bound_2norm=zb)
        assert dz <= 2 * zb
    if p == K and np.array_equal(Ig, o["I"]):
        out["U_rel_err"] = rel(host(g["U"]), o["U"])
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, K, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, K, g["J"], I=g["I"], U=g["U"])
    out.update(residual_id=rid, residual_cur=rcur, ratio_id=rid / o["res"]["id"],
               ratio_cur=rcur / o["res"]["cur"])
    say(name, out)
    assert rid <= 1.05 * o["res"]["id"] and rcur <= 1.05 * o["res"]["cur"]
    return out


def test_poly8192_f32(R, ctx, poly8192, oracle_fp32_values):
    """FP32 mode (FP32 sketch and LUPP on the FP32 values) at the benchmark
    size against the FP64 oracle on the same values."""
    A, Om, o = oracle_fp32_values
    a32, om32 = poly8192
    say("f32 mode", M, N, K, L)
    _low_precision_mode(R, ctx, a32, om32, A, Om, o, "f32")


def test_poly8192_bf16(R, ctx, poly8192):
    """BF16 mode (BF16 storage, BF16 MFMA sketch, FP32 LUPP, FP64 Z with one
    refinement step and U) against the FP64 oracle on the BF16 values."""
    a32, om32 = poly8192
    Ab = a32.T.contiguous().bfloat16().T
    Ob = om32.T.contiguous().bfloat16().T
    A, Om = host(Ab), host(Ob)
    say("oracle on the BF16 values")
    o = O.decompose(A, Om, K, gaps=True)
    o["res"] = O.residuals(A, o["J"], Z=o["Z"], I=o["I"], U=o["U"], only=("id", "cur"))
    say("bf16 mode", M, N, K, L)
    _low_precision_mode(R, ctx, Ab, Ob, A, Om, o, "bf16")


@pytest.mark.parametrize("dt", ["float64", "bfloat16"])
def test_poly8192_overlapped_step_equals_sequential(R, ctx, poly8192, dt):
    """The step as the benchmark times it (Z and the ID residual on a second
    context and stream, beside the CUR step and its residual) at the
    benchmark size: bitwise the J, I, Z and U of the sequential order checked
    against the oracle above, and the residuals of rpid_residual, on every
    repetition."""
    a32, om32 = poly8192
    tdt = getattr(torch, dt)
    Ad = a32.T.contiguous().to(tdt).T
    Od = om32.T.contiguous().to(tdt).T
    say("overlapped step", dt, M, N, K, L)
    ctx2 = R.Context(0, stream=torch.cuda.Stream(device=0))
    try:
        seq = R.decompose(ctx, Ad, Od, K)
        assert seq["status"] == 0 and seq["status_I"] == 0
        rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, K, seq["J"], Z=seq["Z"])
        rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, K, seq["J"], I=seq["I"], U=seq["U"])
        for _ in range(3):
            ov = R.decompose_overlapped(ctx, ctx2, Ad, Od, K)
            assert ov["status"] == 0 and ov["status_I"] == 0
            assert torch.equal(ov["J"], seq["J"]) and torch.equal(ov["I"], seq["I"])
            assert torch.equal(ov["Z"], seq["Z"]) and torch.equal(ov["U"], seq["U"])
            assert ov["residual_id"] == rid and ov["residual_cur"] == rcur
        say("residuals", rid, rcur)
    finally:
        ctx2.close()


def test_lowrank16384_bf16_k512(R, ctx):
    """The BF16 precision form at its own size: 16384 x 16384 stored BF16,
    k = 512, l = 544.  FP32 LUPPs bit-exact against the fixed-arithmetic
    oracle on the kernel's inputs; residuals within 1.05x of the FP64
    oracle's on the stored values; X, Z and U errors printed."""
    m = n = 16384
    k, l = 512, 544
    say("lowrank16384 bf16", m, n, k, l)
    Ab = inputs.torch_lowrank_noise(m, n, k, 1e-4, 9, "cuda").T.contiguous().bfloat16().T
    Ob = inputs.torch_gaussian(l, m, 10, "cuda").T.contiguous().bfloat16().T
    g = R.decompose(ctx, Ab, Ob, k)
    assert g["status"] == 0 and g["status_I"] == 0
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ab, k, g["J"], Z=g["Z"])
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ab, k, g["J"], I=g["I"], U=g["U"])
    Xg, Jg, Ig = host(g["X"]), hint(g["J"]), hint(g["I"])
    Zg, Ug = host(g["Z"]), host(g["U"])
    del g
    A, Om = host(Ab), host(Ob)
    del Ab, Ob
    torch.cuda.empty_cache()
    f = O.lupp_colwise_fma(Xg, k, np.float32)
    assert np.array_equal(Jg, f["J"])
    fr = O.lupp_colwise_fma(A[:, Jg].T, k, np.float32)
    assert np.array_equal(Ig, fr["J"])
    say("oracle (fused LUPPs in float64)")
    o = O.decompose(A, Om, k, lupp="fma")
    res = O.residuals(A, o["J"], Z=o["Z"], I=o["I"], U=o["U"], only=("id", "cur"))
    out = dict(X_rel_err=rel(Xg, o["X"]), J_overlap=len(np.intersect1d(Jg, o["J"])) / k,
               J_prefix=int(np.argmin(Jg == o["J"])) if not np.array_equal(Jg, o["J"]) else k)
    if out["J_prefix"] == k:
        out["Z_rel_err"] = rel(Zg, o["Z"])
        if np.array_equal(Ig, o["I"]):
            out["U_rel_err"] = rel(Ug, o["U"])
    out.update(residual_id=rid, residual_cur=rcur, oracle_id=res["id"], oracle_cur=res["cur"])
    say(out)
    assert np.all(np.abs(Xg - o["X"]) <= 2 * m * U32 * (np.abs(Om) @ np.abs(A)))
    assert rid <= 1.05 * res["id"] and rcur <= 1.05 * res["cur"]


def test_nonneg65536x4096_fp8_cur(R, ctx):
    """The FP8 precision form at its own size: 65536 x 4096 non-negative,
    FP8 sketch (l = 400), FP32 LUPPs, CUR with k = 384.  The LUPPs are
    bit-exact against the fixed-arithmetic oracle on the kernel's inputs, U
    agrees with the oracle's stable U for the same indices, and the CUR
    residual is within 1.05x of the FP64 oracle's own pipeline (its FP8
    sketch accumulated exactly, fused FP64 LUPPs, Householder U)."""
    m, n, r, k, l = 65536, 4096, 384, 384, 400
    say("nonneg65536x4096 fp8", m, n, k, l)
    Ad = inputs.torch_nonneg_lowrank(m, n, r, 1e-3, 5, "cuda")
    Od = inputs.torch_gaussian(l, m, 6, "cuda", dtype=torch.float32)
    Xd = R.rpid_sketch_fp8(ctx, Ad, Od)
    J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, Xd, k)
    assert st == 0
    I, Ud, keff_i, st_i = R.rpid_cur(ctx, Ad, k, J)
    assert st_i == 0
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, J, I=I, U=Ud)
    Xg, Jg, Ig, Ug = host(Xd), hint(J), hint(I), host(Ud)
    Lg, Ugf = host(Lf), host(Uf)
    A, Om = host(Ad), host(Od)
    del Ad, Od, Xd, J, Lf, Uf, I, Ud
    torch.cuda.empty_cache()
    f = O.lupp_colwise_fma(Xg, k, np.float32)
    assert np.array_equal(Jg, f["J"])
    assert np.array_equal(Lg, f["L"].astype(np.float64))
    assert np.array_equal(Ugf, f["U"].astype(np.float64))
    fr = O.lupp_colwise_fma(A[:, Jg].T, k, np.float32)
    assert np.array_equal(Ig, fr["J"])
    Uo_same = O.cur_u(A, Jg, Ig)
    ru = rel(Ug, Uo_same)
    r_same = O.residuals(A, Jg, I=Ig, U=Ug, only=("cur",))["cur"]
    say("U rel err (same indices)", ru, "gpu residual", rcur, "oracle on gpu's U", r_same)
    assert abs(rcur - r_same) <= 1e-6 * r_same
    say("oracle FP8 sketch and pipeline")
    Xo = np.concatenate([O.sketch_fp8(A[:, c:c + 512], Om) for c in range(0, n, 512)], axis=1)
    o = O.decompose(A, Om, k, lupp="fma", X=Xo)
    ro = O.residuals(A, o["J"], I=o["I"], U=o["U"], only=("cur",))["cur"]
    say(dict(X_rel_err=rel(Xg, Xo), J_overlap=len(np.intersect1d(Jg, o["J"])) / k,
             I_overlap=len(np.intersect1d(Ig, o["I"])) / k, residual_cur=rcur, oracle_cur=ro,
             ratio=rcur / ro))
    assert rcur <= 1.05 * ro
