"""GPU test of the overlapped decomposition: Z and the ID residual on a
second context and stream, concurrent with the CUR step, give bitwise the
outputs of the sequential order."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2104_05877_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", ["float64", "bfloat16"])
def test_overlapped_equals_sequential(dt):
    from paper_2104_05877_amd import rpid as R

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print("[overlap]", dt, flush=True)
    m, n, k, l = 2048, 1536, 64, 80
    A, Om = inputs.small_spectral_case(m, n, k, l, inputs.poly_spectrum(min(m, n), 2.0), 31)
    tdt = getattr(torch, dt)
    Ad = inputs.torch_colmajor(A, tdt, "cuda")
    Od = inputs.torch_colmajor(Om, tdt, "cuda")
    ctx = R.Context(0)
    ctx2 = R.Context(0, stream=torch.cuda.Stream(device=0))
    try:
        seq = R.decompose(ctx, Ad, Od, k)
        rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, seq["J"], Z=seq["Z"])
        rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, Ad, k, seq["J"], I=seq["I"], U=seq["U"])
        for _ in range(3):  # repeated, with the side stream reused
            ov = R.decompose_overlapped(ctx, ctx2, Ad, Od, k)
            assert torch.equal(ov["J"], seq["J"]) and torch.equal(ov["I"], seq["I"])
            assert torch.equal(ov["Z"], seq["Z"]) and torch.equal(ov["U"], seq["U"])
            assert ov["residual_id"] == rid and ov["residual_cur"] == rcur
        worker = ctx2.__dict__.get("_side_worker")
    finally:
        ctx2.close()
        ctx.close()
    assert np.isfinite(rid) and np.isfinite(rcur)
    # the side context's worker thread ends with the context
    assert worker is not None and not worker._thread.is_alive()


def test_residual_sums_match_residual():
    """rpid_residual_sums leaves [||A - PQ||^2, ||A||^2] on the device; its
    ratio's square root is bitwise rpid_residual's value."""
    import math

    from paper_2104_05877_amd import rpid as R

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    m, n, k, l = 1024, 768, 32, 40
    A, Om = inputs.small_spectral_case(m, n, k, l, inputs.poly_spectrum(min(m, n), 2.0), 32)
    Ad = inputs.torch_colmajor(A, torch.bfloat16, "cuda")
    Od = inputs.torch_colmajor(Om, torch.bfloat16, "cuda")
    ctx = R.Context(0)
    try:
        d = R.decompose(ctx, Ad, Od, k)
        for which, kw in ((R.RESIDUAL_ID, dict(Z=d["Z"])), (R.RESIDUAL_CUR, dict(I=d["I"], U=d["U"]))):
            r = R.rpid_residual(ctx, which, Ad, k, d["J"], **kw)
            s0, s1 = R.rpid_residual_sums(ctx, which, Ad, k, d["J"], **kw).tolist()
            assert math.sqrt(s0 / s1) == r
    finally:
        ctx.close()


def test_overlapped_zero_pivot_reports_status():
    """A matrix with only 20 nonzero columns and k = 32: the column LUPP meets
    an exactly zero pivot at step 20.  The overlapped step reports the
    sequential call's status and first 20 pivots and returns no
    decomposition; rpid_select_columns_async gives the same pivots and factors
    as rpid_select_columns with the status in a device word, and the work
    enqueued on its J before that word is read (CUR, Z, both residuals, with
    J past step 20 never written) runs to completion without touching memory
    outside its buffers."""
    from paper_2104_05877_amd import rpid as R

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print("[overlap] zero pivot", flush=True)
    m, n, k, l, r = 1024, 768, 32, 40, 20
    rng = np.random.default_rng(41)
    A = np.zeros((m, n))
    cols = rng.choice(n, r, replace=False)
    A[:, cols] = rng.standard_normal((m, r))
    Om = rng.standard_normal((l, m))
    Ad = inputs.torch_colmajor(A, torch.float64, "cuda")
    Od = inputs.torch_colmajor(Om, torch.float64, "cuda")
    ctx = R.Context(0)
    ctx2 = R.Context(0, stream=torch.cuda.Stream(device=0))
    try:
        seq = R.decompose(ctx, Ad, Od, k)
        assert seq["status"] == r + 1 and seq["k_eff"] == r
        for _ in range(2):
            ov = R.decompose_overlapped(ctx, ctx2, Ad, Od, k)
            assert ov["status"] == r + 1 and ov["k_eff"] == r
            assert torch.equal(ov["J"][:r], seq["J"][:r])
            assert "Z" not in ov and "U" not in ov
        # the asynchronous pivots, and dependent work on them, before the status is read
        for dt in (torch.float64, torch.float32):
            X = R.rpid_sketch(ctx, Ad.to(dt), Od.to(dt))
            Js, Ls, Us, ds, ke, st = R.rpid_select_columns(ctx, X, k)
            Ja, La, Ua, da, st_dev = R.rpid_select_columns_async(ctx, X, k)
            # J past step 20 is unwritten: breakdown statuses from the garbage
            # are expected, faults are not
            try:
                I, U, ke_i, st_i = R.rpid_cur(ctx, Ad, k, Ja)
                R.rpid_residual_sums(ctx, R.RESIDUAL_CUR, Ad, k, Ja, I=I, U=U)
            except R.RpidError:
                pass
            try:
                Z, _ = R.rpid_id_coeffs(ctx, X, k, Ja, La, Ua)
                R.rpid_residual_sums(ctx, R.RESIDUAL_ID, Ad, k, Ja, Z=Z)
            except R.RpidError:
                pass
            torch.cuda.synchronize()
            assert int(st_dev.item()) == st == r + 1
            assert torch.equal(Ja[:r], Js[:r]) and torch.equal(La[:, :r], Ls[:, :r])
            assert torch.equal(Ua[:r, :r], Us[:r, :r])
        # the contexts still work afterwards
        A2, Om2 = inputs.small_spectral_case(m, n, k, l, inputs.poly_spectrum(min(m, n), 2.0), 42)
        ok = R.decompose_overlapped(ctx, ctx2, inputs.torch_colmajor(A2, torch.float64, "cuda"),
                                    inputs.torch_colmajor(Om2, torch.float64, "cuda"), k)
        assert ok["status"] == 0 and np.isfinite(ok["residual_id"]) and np.isfinite(ok["residual_cur"])
    finally:
        ctx2.close()
        ctx.close()
