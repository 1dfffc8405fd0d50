"""Pins of the FP64 learned-rank oracle against facts that do not come from
the oracle itself: finite differences, closed-form networks, closed-form
Adam and loss values, exact-rank matrices (Lemma 1).  CPU only."""
from __future__ import annotations

import types

import numpy as np
import pytest

import oracle.mlp_oracle as M
from paper_2104_05877_amd import inputs


def _rand_params(rng, scale=0.1):
    return rng.standard_normal(M.NPARAM) * scale


def pin_fd_gradient(Mo, seed=1, B=5):
    """Analytic gradient of the pinball loss through the network equals
    central differences on a sample of parameters of every block."""
    rng = np.random.default_rng(seed)
    W = _rand_params(rng, 0.2)
    X = rng.standard_normal((B, Mo.IN))
    t = rng.standard_normal(B)
    y, cache = Mo.forward(W, X)
    _, dy = Mo.pinball(y, t, 0.9)
    g = Mo.backward(W, X, cache, dy)
    idx = np.concatenate([rng.integers(lo, hi, 6) for lo, hi in (
        (Mo.OFF_W1, Mo.OFF_B1), (Mo.OFF_B1, Mo.OFF_W2), (Mo.OFF_W2, Mo.OFF_B2),
        (Mo.OFF_B2, Mo.OFF_W3), (Mo.OFF_W3, Mo.OFF_B3))] + [[Mo.OFF_B3]])
    h = 1e-6
    for p in idx:
        Wp, Wm = W.copy(), W.copy()
        Wp[p] += h
        Wm[p] -= h
        lp = Mo.pinball(Mo.forward(Wp, X)[0], t, 0.9)[0]
        lm = Mo.pinball(Mo.forward(Wm, X)[0], t, 0.9)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 + 1e-4 * abs(fd), (p, fd, g[p])


def pin_identity_network(Mo, seed=2):
    """Hidden units relu(x_3) and relu(-x_3), passed through, output
    difference: the network computes x_3 + b3 exactly."""
    W1 = np.zeros((Mo.H, Mo.IN))
    W1[0, 3], W1[1, 3] = 1.0, -1.0
    W2 = np.zeros((Mo.H, Mo.H))
    W2[5, 0], W2[9, 1] = 1.0, 1.0
    w3 = np.zeros(Mo.H)
    w3[5], w3[9] = 1.0, -1.0
    W = Mo.pack(W1, np.zeros(Mo.H), W2, np.zeros(Mo.H), w3, 0.25)
    X = np.random.default_rng(seed).standard_normal((7, Mo.IN))
    y, _ = Mo.forward(W, X)
    assert np.allclose(y, X[:, 3] + 0.25, rtol=0, atol=1e-15)


def pin_homogeneity(Mo, seed=3):
    """With zero biases a ReLU network is positively homogeneous."""
    rng = np.random.default_rng(seed)
    W1, _, W2, _, w3, _ = Mo.unpack(_rand_params(rng))
    W = Mo.pack(W1, np.zeros(Mo.H), W2, np.zeros(Mo.H), w3, 0.0)
    X = rng.standard_normal((4, Mo.IN))
    y1, _ = Mo.forward(W, X)
    y3, _ = Mo.forward(W, 3.0 * X)
    assert np.allclose(y3, 3.0 * y1, rtol=1e-12, atol=1e-14)
    yn, _ = Mo.forward(W, -X)
    assert not np.allclose(yn, -y1)  # ReLU is not odd


def pin_pinball(Mo):
    """r = 2 (under-prediction) costs tau * 2; r = -2 costs (1 - tau) * 2."""
    loss, dy = Mo.pinball(np.array([0.0, 4.0]), np.array([2.0, 2.0]), 0.9)
    assert abs(loss - (0.9 * 2 + 0.1 * 2) / 2) < 1e-15
    assert np.allclose(dy, [-0.9 / 2, 0.1 / 2])


def pin_adam_first_step(Mo):
    """First step with zero moments moves every parameter by lr*sign(g)
    (up to eps): m_hat = g, v_hat = g^2."""
    g = np.array([0.5, -2.0, 1e-3])
    W1, m1, m2 = Mo.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 0.01, 1)
    assert np.allclose(W1, -0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def pin_features(Mo):
    f = Mo.features(np.array([2.0, 0.2, 0.02, 2e-30, 1.0]), 6, 4)
    assert np.allclose(f, [0.0, -1.0, -2.0, -20.0, -20.0, -20.0], atol=1e-12)


def pin_label_exact_rank(Mo, seed=4, m=90, n=70, r=9, l=20):
    """rank(A) = r: rank r reproduces A (Lemma 1), rank r - 1 cannot."""
    A, Om = inputs.small_spectral_case(m, n, r, l, np.linspace(1.0, 0.5, r), seed)
    assert Mo.rank_label(A, Om, 1e-10, l) == r


def pin_label_sandwich(Mo, seed=5, m=120, n=100, l=40, tol=1e-4):
    """The label is the first rank whose residual reaches tol."""
    A, Om = inputs.small_spectral_case(m, n, l, l, inputs.exp_spectrum(min(m, n), 20.0), seed)
    k = Mo.rank_label(A, Om, tol, l)
    assert k is not None and k > 1
    from oracle import rpid_oracle as O

    Xs = O.sketch(A, Om)
    J = O.lupp_colwise(Xs, l)["J"]
    assert Mo.id_residual_at(A, Xs, J, k) <= tol < Mo.id_residual_at(A, Xs, J, k - 1)


PINS = [pin_fd_gradient, pin_identity_network, pin_homogeneity, pin_pinball,
        pin_adam_first_step, pin_features, pin_label_exact_rank, pin_label_sandwich]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin(M)


MUTANTS = {
    "backward without the ReLU mask": ("dz2 = np.outer(dy, w3) * (z2 > 0)", "dz2 = np.outer(dy, w3)"),
    "W2 transposed in forward": ("z2 = h1 @ W2.T + b2", "z2 = h1 @ W2 + b2"),
    "pinball gradient sign": ("dy = np.where(r > 0, -tau,", "dy = np.where(r > 0, tau,"),
    "Adam without bias correction": ("mh = m1 / (1 - b1**t)", "mh = m1"),
    "natural log features": ("f[t] = max(np.log10(r), -20.0)", "f[t] = max(np.log(r), -20.0)"),
    "label one rank late": ("            return k\n    return None", "            return k + 1\n    return None"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mlp_oracle_mutants_are_caught(name):
    old, new = MUTANTS[name]
    src = open(M.__file__).read()
    assert old in src, name
    mod = types.ModuleType("mlp_oracle_mutant")
    exec(compile(src.replace(old, new), "mlp_oracle_mutant", "exec"), mod.__dict__)
    caught = False
    for pin in PINS:
        try:
            pin(mod)
        except AssertionError:
            caught = True
            break
    assert caught, f"no pin catches mutant {name!r}"
