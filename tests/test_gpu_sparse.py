"""GPU tests of the sparse and structured sketches against the FP64 oracle:
the sparse sign embedding on a dense A, the CSC sketch of a sparse A (dense
Gaussian or sparse sign embedding), CSC column gathering, and Rand-LUPP end
to end on an SNN matrix (eq. snn-def) of the size the paper uses."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.rpid_oracle as O  # noqa: E402
from paper_2104_05877_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print("[sparse]", *a, flush=True)


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


def dev(a, dt=torch.float64):
    return inputs.torch_colmajor(a, dt, "cuda")


def snn1e3(seed, rho=0.01):
    """SNN1e3 of Sec. 5: 1000 x 1000, r = 1000, s_i = 2/i (i <= 100), 1/i after."""
    i = np.arange(1, 1001, dtype=np.float64)
    s = np.where(i <= 100, 2.0 / i, 1.0 / i)
    return inputs.snn_csc(np.random.default_rng(seed), 1000, 1000, s, rho)


def to_dev_csc(R, colptr, rowidx, vals, m, n, dt=torch.float64):
    return R.CSC(torch.from_numpy(colptr).cuda(), torch.from_numpy(rowidx).cuda(),
                 torch.from_numpy(vals).to(dt).cuda(), m, n)


@pytest.mark.parametrize("m,n,l,zeta,seed", [(1000, 800, 60, 8, 1), (777, 640, 40, 3, 2), (4096, 2048, 272, 8, 3)])
@pytest.mark.parametrize("dt", ["float64", "float32", "bfloat16"])
def test_sparse_sign_dense_against_oracle(R, ctx, m, n, l, zeta, seed, dt):
    """|X - scale S A| <= 2 (m + 2) u scale |S| |A| on the stored values (the
    +-1 entries are exact in every storage type)."""
    say("sparse sign dense", dt, m, n, l, zeta)
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    rows, signs = inputs.sparse_sign_draws(rng, m, l, zeta)
    scale = 1.0 / np.sqrt(zeta)
    Ad = dev(A, getattr(torch, dt))
    a_s = host(Ad)
    X = R.rpid_sketch_sparse_sign(ctx, Ad, torch.from_numpy(rows).cuda(), torch.from_numpy(signs).cuda(), l, scale)
    ref = O.sketch_sparse_sign(a_s, rows, signs, l, scale)
    u = 2.0**-53 if dt == "float64" else 2.0**-24
    S = np.abs(O.sparse_sign_matrix(rows, signs, l))
    bound = 2 * (m + 2) * u * scale * (S @ np.abs(a_s)) + 1e-300
    err = np.abs(host(X) - ref)
    say("max err/bound", float((err / bound).max()))
    assert np.all(err <= bound)


@pytest.mark.parametrize("dt", ["float64", "float32"])
def test_csc_sketch_against_oracle(R, ctx, dt):
    """Gaussian and sparse sign sketches of SNN1e3 (about 9.5 % nonzeros) and
    of a 3000 x 2000 matrix with 0.2 % nonzeros and empty columns, against
    the oracle on the stored values; CSC gathering equals the dense columns."""
    tdt = getattr(torch, dt)
    u = 2.0**-53 if dt == "float64" else 2.0**-24
    rng = np.random.default_rng(4)
    cases = [(snn1e3(5), 1000, 1000)]
    m2, n2 = 3000, 2000
    cp, ri, va = inputs.snn_csc(rng, m2, n2, np.array([1.0, 0.5, 0.25]), 0.03)
    cases.append(((cp, ri, va), m2, n2))
    for (colptr, rowidx, vals), m, n in cases:
        A = to_dev_csc(R, colptr, rowidx, vals, m, n, tdt)
        v_s = host(A.vals)
        Ad = O.csc_dense(colptr, rowidx, v_s, m, n)
        say("csc", dt, m, n, "nnz", A.nnz, "empty columns", int(np.sum(np.diff(colptr) == 0)))
        for l in (64, 300):
            G = rng.standard_normal((l, m))
            Gd = dev(G, tdt)
            X = R.rpid_sketch_csc(ctx, A, Gd)
            ref = O.sketch_csc(colptr, rowidx, v_s, m, n, host(Gd))
            bound = 2 * (m + 2) * u * (np.abs(host(Gd)) @ np.abs(Ad)) + 1e-300
            assert np.all(np.abs(host(X) - ref) <= bound)
            rows, signs = inputs.sparse_sign_draws(rng, m, l, 8)
            Xs = R.rpid_sketch_csc_sparse_sign(ctx, A, torch.from_numpy(rows).cuda(),
                                               torch.from_numpy(signs).cuda(), l, 0.5)
            refs = O.sketch_sparse_sign(Ad, rows, signs, l, 0.5)
            bounds = 2 * (m + 2) * u * 0.5 * (np.abs(O.sparse_sign_matrix(rows, signs, l)) @ np.abs(Ad)) + 1e-300
            assert np.all(np.abs(host(Xs) - refs) <= bounds)
        J = torch.tensor([0, n - 1, 7, 3, 7], dtype=torch.int64, device="cuda")
        C = R.rpid_csc_gather(ctx, A, J)
        assert np.array_equal(host(C), Ad[:, [0, n - 1, 7, 3, 7]])
        assert np.array_equal(host(R.rpid_csc_gather(ctx, A)), Ad)


@pytest.mark.parametrize("embedding", ["gaussian", "sparse_sign"])
def test_snn1e3_rand_lupp(R, ctx, embedding):
    """Rand-LUPP on SNN1e3 from the CSC sketch (FP64): J equals the oracle's
    on the same sketch values up to the first near-tie, and the ID residual
    (computed on the densified matrix) is within 1e-9 of the oracle's."""
    colptr, rowidx, vals = snn1e3(6)
    m = n = 1000
    k, l = 50, 60
    A = to_dev_csc(R, colptr, rowidx, vals, m, n)
    Ad = O.csc_dense(colptr, rowidx, vals, m, n)
    rng = np.random.default_rng(7)
    if embedding == "gaussian":
        G = rng.standard_normal((l, m))
        X = R.rpid_sketch_csc(ctx, A, dev(G))
        Xo = G @ Ad
    else:
        rows, signs = inputs.sparse_sign_draws(rng, m, l, 8)
        X = R.rpid_sketch_csc_sparse_sign(ctx, A, torch.from_numpy(rows).cuda(), torch.from_numpy(signs).cuda(),
                                          l, 1.0 / np.sqrt(8))
        Xo = O.sketch_sparse_sign(Ad, rows, signs, l, 1.0 / np.sqrt(8))
    J, Lf, Uf, _, keff, st = R.rpid_select_columns(ctx, X, k)
    assert st == 0
    f = O.lupp_colwise(host(X), k, gaps=True)
    fc = int(np.argmax(f["gap"] < 1e-9)) if (f["gap"] < 1e-9).any() else k
    assert np.array_equal(J.cpu().numpy()[:fc], f["J"][:fc])
    Z, _ = R.rpid_id_coeffs(ctx, X, k, J, Lf, Uf)
    Adev = R.rpid_csc_gather(ctx, A)
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Adev, k, J, Z=Z)
    fo = O.lupp_colwise(Xo, k)
    ro = O.residuals(Ad, fo["J"], Z=O.id_coeffs(Xo, fo["J"], k), only=("id", "idopt"))
    say(embedding, "snn1e3 id residual gpu", rid, "oracle", ro["id"], "optimal-C", ro["idopt"], "matched", fc)
    if fc == k:
        assert abs(rid - ro["id"]) <= 1e-9 * ro["id"]
    else:
        assert rid <= 1.05 * ro["id"]


def test_sparse_argument_errors(R, ctx):
    A = dev(np.zeros((64, 32)))
    rows = torch.zeros((64, 9), dtype=torch.int32, device="cuda")
    signs = torch.ones((64, 9), dtype=torch.int8, device="cuda")
    with pytest.raises(R.RpidError) as e:  # zeta > l
        R.rpid_sketch_sparse_sign(ctx, A, rows, signs, 8, 1.0)
    assert e.value.status == -9
    with pytest.raises(ValueError):
        R.rpid_sketch_sparse_sign(ctx, A, rows.long(), signs, 16, 1.0)
    with pytest.raises(R.RpidError) as e:  # non-positive scale
        R.rpid_sketch_sparse_sign(ctx, A, rows, signs, 16, 0.0)
    assert e.value.status == -11


@pytest.mark.parametrize("m,n,l,seed", [(1024, 700, 64, 11), (1000, 513, 100, 12)])
@pytest.mark.parametrize("dt", ["float64", "float32", "bfloat16"])
def test_srtt_against_oracle(R, ctx, m, n, l, seed, dt):
    """The SRTT sketch (DHT, random permutation, signs and row selection)
    against the oracle's explicit Gamma = sqrt(m/l) S T Phi P on the stored
    A: within (2m + 8) u |Gamma| |A|, plus 2^-8 |Gamma| |A| in BF16, whose
    embedding entries are rounded to BF16."""
    say("srtt", dt, m, n, l)
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    perm, phi, sel = inputs.srtt_draws(rng, m, l)
    Ad = dev(A, getattr(torch, dt))
    a_s = host(Ad)
    X = R.rpid_sketch_srtt(ctx, Ad, torch.from_numpy(perm).cuda(), torch.from_numpy(phi).cuda(),
                           torch.from_numpy(sel).cuda())
    G = O.srtt_matrix(perm, phi, sel, m, l)
    ref = G @ a_s
    u = 2.0**-53 if dt == "float64" else 2.0**-24
    mag = np.abs(G) @ np.abs(a_s)
    bound = (2 * m + 8) * u * mag + (2.0**-8 * mag if dt == "bfloat16" else 0.0) + 1e-300
    err = np.abs(host(X) - ref)
    say("max err/bound", float((err / bound).max()))
    assert np.all(err <= bound)


def test_srtt_rand_lupp_fp64(R, ctx):
    """Rand-LUPP on an SRTT sketch (FP64): pivots equal the oracle's on the
    same sketch values up to the first near-tie and the ID residual matches
    to 1e-9 relative."""
    m, n, k, l = 1024, 900, 40, 50
    A, _ = inputs.small_spectral_case(m, n, k, l, inputs.poly_spectrum(min(m, n), 2.0), 13)
    perm, phi, sel = inputs.srtt_draws(np.random.default_rng(14), m, l)
    Ad = dev(A)
    X = R.rpid_sketch_srtt(ctx, Ad, torch.from_numpy(perm).cuda(), torch.from_numpy(phi).cuda(),
                           torch.from_numpy(sel).cuda())
    J, Lf, Uf, _, keff, st = R.rpid_select_columns(ctx, X, k)
    assert st == 0
    f = O.lupp_colwise(host(X), k, gaps=True)
    fc = int(np.argmax(f["gap"] < 1e-9)) if (f["gap"] < 1e-9).any() else k
    assert np.array_equal(J.cpu().numpy()[:fc], f["J"][:fc])
    Z, _ = R.rpid_id_coeffs(ctx, X, k, J, Lf, Uf)
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, Ad, k, J, Z=Z)
    Xo = O.sketch_srtt(A, perm, phi, sel, l)
    fo = O.lupp_colwise(Xo, k)
    ro = O.residuals(A, fo["J"], Z=O.id_coeffs(Xo, fo["J"], k), only=("id",))["id"]
    say("srtt id residual gpu", rid, "oracle", ro, "matched", fc)
    if fc == k:
        assert abs(rid - ro) <= 1e-9 * ro
    else:
        assert rid <= 1.05 * ro


@pytest.mark.parametrize("dt", ["float64", "float32"])
@pytest.mark.parametrize("zeta,l", [(8, 300), (3, 64), (1, 17), (64, 64), (8, 1024)])
def test_csc_sparse_sign_direct_is_the_expanded_product(R, ctx, dt, zeta, l):
    """The sparse sign embedding applied as a sparse operator to a CSC matrix
    gives, bit for bit, the CSC sketch with the same embedding written out
    densely (each term +-a_ij exact, the terms of a row added in the storage
    order of the column, the scale applied once), the same bits on a second
    call, and lies within 2(m + 2)u scale |S||A| of the oracle.  SNN1e3 and a
    3000 x 2000 matrix with empty columns (n not a multiple of the columns a
    wave takes); zeta from 1 to 64 (one nonzero per wave round); l up to
    1024 (the largest LDS footprint)."""
    tdt = getattr(torch, dt)
    u = 2.0**-53 if dt == "float64" else 2.0**-24
    rng = np.random.default_rng(40 + zeta)
    cases = [(snn1e3(31), 1000, 1000)]
    A2 = np.zeros((3000, 2000))
    mask = rng.random((3000, 2000)) < 0.002
    A2[mask] = rng.standard_normal(int(mask.sum()))
    A2[:, ::7] = 0.0
    from scipy.sparse import csc_matrix

    sp = csc_matrix(A2)
    sp.sort_indices()
    cases.append(((sp.indptr.astype(np.int64), sp.indices.astype(np.int64), sp.data.astype(np.float64)), 3000,
                  2000))
    for (cp, ri, va), m, n in cases:
        say("csc sparse sign direct", dt, m, n, "nnz", len(va), "zeta", zeta, "l", l)
        A = to_dev_csc(R, cp, ri, va, m, n, tdt)
        rows, signs = inputs.sparse_sign_draws(rng, m, l, zeta)
        scale = 1.0 / np.sqrt(zeta)
        rd, sd = torch.from_numpy(rows).cuda(), torch.from_numpy(signs).cuda()
        X1 = R.rpid_sketch_csc_sparse_sign(ctx, A, rd, sd, l, scale)
        X2 = R.rpid_sketch_csc_sparse_sign(ctx, A, rd, sd, l, scale)
        S = O.sparse_sign_matrix(rows, signs, l)
        Xe = R.rpid_sketch_csc(ctx, A, dev(S, tdt)) * torch.tensor(scale, dtype=tdt)
        torch.cuda.synchronize()
        assert torch.equal(X1, X2)
        Ad = O.csc_dense(cp, ri, host(A.vals), m, n)
        ref = O.sketch_sparse_sign(Ad, rows, signs, l, scale)
        bound = 2 * (m + 2) * u * scale * (np.abs(S) @ np.abs(Ad)) + 1e-300
        assert np.all(np.abs(host(X1) - ref) <= bound)
        assert torch.equal(X1, Xe), float((X1 - Xe).abs().max())
