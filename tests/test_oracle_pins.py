"""The FP64 oracle against what the paper and the mathematics fix (CPU)."""
import types

import numpy as np
import pytest

import oracle.rpid_oracle as O
from tests import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(O)


def test_nonfinite_rejected():
    X = np.ones((3, 5))
    X[1, 2] = np.nan
    with pytest.raises(O.NonFiniteInput):
        O.lupp_colwise(X, 3)


def test_exp1000x800_floor():
    """The exponential workload's optimal rank-50 relative error is a closed
    form of its spectrum (Eckart-Young); the oracle's optimal-ID and sketch-ID
    errors sit at or above it, and the generator realises the spectrum."""
    from paper_2104_05877_amd import inputs

    s = inputs.exp_spectrum(800, 8.0)
    assert abs(O.optimal_error(s, 50) - 0.3158) < 5e-5
    a, om, k, l = inputs.case_exp1000x800()
    sv = np.linalg.svd(a, compute_uv=False)
    np.testing.assert_allclose(sv, s, rtol=1e-9, atol=1e-15)
    d = O.decompose(a, om, k)
    r = O.residuals(a, d["J"], Z=d["Z"], I=d["I"], U=d["U"])
    assert O.optimal_error(s, k) <= r["idopt"] <= r["id"]
    assert r["idopt"] <= r["cur"]


MUTANTS = {
    "argmax without modulus": ("cand = np.abs(S[:, t])", "cand = S[:, t].copy()"),
    "Schur update sign": ("-= np.outer(mult, S[p, t + 1 : k])", "+= np.outer(mult, S[p, t + 1 : k])"),
    "ties to largest index": ("p = int(np.argmax(cand))", "p = int(len(cand) - 1 - np.argmax(cand[::-1]))"),
    "multiplier from wrong pivot": ("mult = S[remaining, t] / piv", "mult = S[remaining, t] / S[p, min(t + 1, k - 1)]"),
    "U row stored as column": ("U[t, t:] = S[p, t:]", "U[t:, t] = S[p, t:]"),
    "Z with transposed X_1": ("Z = np.linalg.solve(Xk[:, J], Xk)", "Z = np.linalg.solve(Xk[:, J].T, Xk)"),
    "U right factor on the left": (
        "U = sla.solve_triangular(rr, U.T, lower=False).T",
        "U = sla.solve_triangular(rr, U, lower=False)",
    ),
    "eta without the identity block": ("return float(np.sqrt(1.0 + s * s))", "return float(np.sqrt(s * s))"),
    "id residual not relative": ('out["id"] = nrm(A - C @ _f64(Z)) / na', 'out["id"] = nrm(A - C @ _f64(Z))'),
    "CUR with R transposed factor": ('qr_, rr = np.linalg.qr(R.T)', 'qr_, rr = np.linalg.qr(R.T[:, ::-1])'),
    "E4M3 ties away from zero": ("pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))",
                                 "pick_hi = (dhi <= dlo)"),
    "FP8 scale one step high": ("    while np.ldexp(mx, e) > E4M3_MAX:\n        e -= 1\n    return e",
                                "    while np.ldexp(mx, e) > E4M3_MAX:\n        e -= 1\n    return e + 1"),
    "FP8 sketch not unscaled": ("return (Oq @ Aq) * np.ldexp(1.0, -(eo + ea))[None, :]", "return Oq @ Aq"),
    "power sketch with a second power": ("    Y = A @ _f64(Omega).T\n    return Y.T @ A",
                                         "    Y = A @ _f64(Omega).T\n    return (Y.T @ A) @ (A.T @ A)"),
    "power sketch normalised": ("    Y = A @ _f64(Omega).T\n    return Y.T @ A",
                                "    Y = A @ _f64(Omega).T\n    return Y.T @ A / np.linalg.norm(A)"),
    "two-sided Y with the columns of Omega reversed": ("return _f64(Gamma) @ A, A @ _f64(Omega).T",
                                                   "return _f64(Gamma) @ A, A @ _f64(Omega)[:, : A.shape[1]].T[::-1]"),
    "row ID from the untransposed system": ("W = np.linalg.solve(Yk[I, :].T, Yk.T).T",
                                            "W = np.linalg.solve(Yk[I, :], Yk.T).T"),
    "cheap CUR core not inverted": ("return np.linalg.solve(S, np.eye(S.shape[0]))", "return S"),
    "cheap CUR core from S transposed": ("return np.linalg.solve(S, np.eye(S.shape[0]))",
                                         "return np.linalg.solve(S.T, np.eye(S.shape[0]))"),
    "CPQR norms over all rows": ("norms = np.sqrt(np.sum(S[t:, :] ** 2, axis=0))",
                                 "norms = np.sqrt(np.sum(S ** 2, axis=0))"),
    "CPQR ties to the largest column": ("p = int(cand.argmax())  # the first maximum",
                                        "p = int(len(cand) - 1 - cand[::-1].argmax())"),
    "CPQR reflector sign flipped": ("alpha = -np.linalg.norm(w) if w[0] >= 0.0 else np.linalg.norm(w)",
                                    "alpha = np.linalg.norm(w) if w[0] >= 0.0 else -np.linalg.norm(w)"),
    "CPQR update without beta": ("S[t:, cols] -= beta * np.outer(v, d)", "S[t:, cols] -= np.outer(v, d)"),
    "CPQR Z from the transposed R_11": ("Z = sla.solve_triangular(R[:k, J], R[:k, :], lower=False)",
                                        "Z = sla.solve_triangular(R[:k, J].T, R[:k, :], lower=True)"),
    "sparse sign entry at the wrong row": ("            G[rows[i, s_], i] = float(signs[i, s_])",
                                           "            G[(rows[i, s_] + 1) % l, i] = float(signs[i, s_])"),
    "sparse sign sketch without the scale": ("return float(scale) * (sparse_sign_matrix(rows, signs, l) @ _f64(A))",
                                             "return sparse_sign_matrix(rows, signs, l) @ _f64(A)"),
    "CSC entries transposed": ("            A[int(rowidx[p]), j] = float(vals[p])",
                               "            A[int(rowidx[p]) % n, j % m] = float(vals[p])"),
    "DHT with cos - sin": ("return (np.cos(ang) + np.sin(ang)) / np.sqrt(m)", "return (np.cos(ang) - np.sin(ang)) / np.sqrt(m)"),
    "SRTT permutation applied inverted": ("P[np.arange(m), np.asarray(perm)] = 1.0", "P[np.asarray(perm), np.arange(m)] = 1.0"),
    "least-squares Z over the first k rows only": ("    Z = np.linalg.lstsq(X[:, J], X, rcond=None)[0]",
                                                    "    Z = np.linalg.lstsq(X[:k][:, J], X[:k], rcond=None)[0]"),
    "rangefinder projected on the row space of all l rows": ("    q, _ = np.linalg.qr(_f64(X)[:k, :].T)",
                                                              "    q, _ = np.linalg.qr(_f64(X).T)"),
    "rangefinder error of the projection instead of the remainder": (
        "    E = A - (A @ q) @ q.T", "    E = (A @ q) @ q.T"),
    "row ID residual with C instead of R": ('out["rowid"] = nrm(A - _f64(W) @ R) / na',
                                            'out["rowid"] = nrm(A - _f64(W) @ R[:, ::-1]) / na'),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_oracle_mutants_are_caught(name):
    """A plausible mistake planted in the oracle (on the CPU) fails a pin."""
    old, new = MUTANTS[name]
    src = open(O.__file__).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle_mutant")
    mod.__file__ = O.__file__
    exec(compile(src.replace(old, new), "oracle_mutant", "exec"), mod.__dict__)
    caught = []
    for pin in P.ALL_PINS:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except Exception as e:  # noqa: BLE001  (assertion or numerical failure)
            caught.append((pin.__name__, type(e).__name__))
    assert caught, f"no pin catches mutant {name!r}"
