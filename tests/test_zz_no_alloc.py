"""The allocation-free sketch entry point (rpid_sketch_noalloc) against
rpid_sketch, through the C-ABI: two calls in a row on the fixed device
scratch, the second on a smaller input, in every supported type.  Where
rpid_sketch's split-K count fits the scratch the two results must be
bitwise equal (same kernels, same summation order); at the largest FP64
benchmark size the split is capped and X must stay within the FP64
accumulation bound of rpid_sketch's X.  Oversized inputs are refused
before anything is enqueued."""
from __future__ import annotations

import ctypes

import pytest

torch = pytest.importorskip("torch")

from paper_2104_05877_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

RPID_ERR_SCRATCH = -107


def say(*a):
    print("[no-alloc]", *a, flush=True)


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


def operands(m, n, l, dtype, seed):
    A = inputs.torch_gaussian(m, n, seed, "cuda").T.contiguous().to(dtype).T
    Om = inputs.torch_gaussian(l, m, seed + 1, "cuda").T.contiguous().to(dtype).T
    return A, Om


def out_like(R, l, n, dtype):
    xt = torch.float32 if dtype == torch.bfloat16 else dtype
    return R.empty_colmajor(l, n, xt, "cuda")


CASES = {
    # (m, n, l) of the first call, then of the second (smaller) call; every
    # size keeps rpid_sketch's own split-K partials inside the 64 MiB scratch
    "f64": (torch.float64, (3000, 1000, 200), (777, 513, 50)),
    "f32": (torch.float32, (4096, 2048, 272), (1000, 300, 64)),
    "bf16": (torch.bfloat16, (8192, 8192, 272), (2048, 1024, 136)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_noalloc_matches_sketch_twice(R, ctx, name):
    dtype, big, small = CASES[name]
    ops = [operands(*big, dtype, 11), operands(*small, dtype, 21)]
    outs = []
    for (A, Om), (m, n, l) in zip(ops, (big, small)):
        say(name, "noalloc call", m, n, l)
        X = out_like(R, l, n, dtype)
        X.fill_(float("nan"))
        outs.append(R.rpid_sketch_noalloc(ctx, A, Om, X))
    torch.cuda.synchronize()
    for (A, Om), Xn, shape in zip(ops, outs, (big, small)):
        Xr = R.rpid_sketch(ctx, A, Om)
        torch.cuda.synchronize()
        assert torch.isfinite(Xn).all(), shape
        assert torch.equal(Xn, Xr), (name, shape, float((Xn - Xr).abs().max()))
        say(name, shape, "bitwise equal to rpid_sketch")


def test_noalloc_capped_split_within_bound(R, ctx):
    """8192 x 8192 FP64 with l = 272: the packed Omega^T (17.8 MB) leaves
    room for fewer split-K slices than rpid_sketch takes, so only the
    summation order differs: |X_noalloc - X| <= 2 m u |Omega| |A|."""
    m = n = 8192
    l = 272
    A, Om = operands(m, n, l, torch.float64, 31)
    X = out_like(R, l, n, torch.float64)
    say("f64 capped split", m, n, l)
    R.rpid_sketch_noalloc(ctx, A, Om, X)
    Xr = R.rpid_sketch(ctx, A, Om)
    bound = 2 * m * 2.0**-53 * (Om.abs() @ A.abs())
    torch.cuda.synchronize()
    assert bool(((X - Xr).abs() <= bound).all())
    # and a smaller call right after it still matches bitwise
    A2, Om2 = operands(1024, 777, 64, torch.float64, 41)
    X2 = out_like(R, 64, 777, torch.float64)
    R.rpid_sketch_noalloc(ctx, A2, Om2, X2)
    assert torch.equal(X2, R.rpid_sketch(ctx, A2, Om2))


def test_noalloc_refuses_oversized_input(R, ctx):
    """m l e_A beyond the scratch is refused before anything is enqueued (the
    pointers are never read), and the context keeps working."""
    A, Om = operands(64, 64, 16, torch.float64, 51)
    X = out_like(R, 16, 64, torch.float64)
    m_big = 40000  # 40000 x 272 FP64 = 87 MB of packed Omega^T
    s = R.lib().rpid_sketch_noalloc(ctx.handle, ctypes.c_void_p(A.data_ptr()), R.F64, m_big, 64, m_big,
                                    ctypes.c_void_p(Om.data_ptr()), R.F64, 272, 272,
                                    ctypes.c_void_p(X.data_ptr()), R.F64, 272)
    assert s == RPID_ERR_SCRATCH
    assert R.lib().rpid_status_string(s).startswith(b"input larger than the fixed scratch")
    R.rpid_sketch_noalloc(ctx, A, Om, X)
    assert torch.equal(X, R.rpid_sketch(ctx, A, Om))
