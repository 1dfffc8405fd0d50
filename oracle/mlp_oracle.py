"""FP64 CPU oracle for the learned-rank form (not in the paper).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module: only the tests use it.  It shares no code with the HIP path.

What it computes:

* features        -- the pivot-magnitude profile of a sketch's LUPP,
                     f_t = max(log10(|u_tt| / |u_00|), -20) for t < k_eff and
                     -20 after an exact zero pivot (|u_tt| are the pivots of
                     eq. (def_LUPP));
* forward/backward-- the network 512 -> 128 -> 128 -> 1 with ReLU on both
                     hidden layers, parameters in one flat vector
                     [W1 (128 x 512 row-major), b1, W2 (128 x 128), b2, w3, b3];
                     backward returns d(sum_b dy_b y_b)/dW;
* pinball         -- quantile loss at level tau on r = target - y (mean);
* adam            -- one Adam step (0.9, 0.999, 1e-8) with bias correction;
* rank_label      -- the smallest k <= lmax whose sketch-based ID (Sec. 4,
                     Alg. 2 with the first k pivots) has relative Frobenius
                     residual <= tol, by scanning every k (brute force); None
                     when no k <= lmax meets tol.

Reading taken: the residual at rank k uses the first k pivots and the first
k rows of the l-row sketch (prefix property of LUPP), i.e. exactly what the
plain path computes when asked for rank k.
"""
from __future__ import annotations

import numpy as np

from oracle import rpid_oracle as O

IN, H = 512, 128
OFF_W1 = 0
OFF_B1 = H * IN
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
NPARAM = OFF_B3 + 1


def unpack(W):
    W = np.asarray(W, dtype=np.float64)
    return (W[OFF_W1:OFF_B1].reshape(H, IN), W[OFF_B1:OFF_W2], W[OFF_W2:OFF_B2].reshape(H, H),
            W[OFF_B2:OFF_W3], W[OFF_W3:OFF_B3], W[OFF_B3])


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def features(diag, L, k_eff):
    """f_t = max(log10(diag[t] / diag[0]), -20) for t < k_eff, else -20."""
    diag = np.asarray(diag, dtype=np.float64)
    f = np.full(L, -20.0)
    for t in range(min(L, k_eff)):
        r = diag[t] / diag[0]
        if r > 0:
            f[t] = max(np.log10(r), -20.0)
    return f


def forward(W, X):
    """y (B,) and the cache (z1, h1, z2, h2) for backward."""
    W1, b1, W2, b2, w3, b3 = unpack(W)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (z1, h1, z2, h2)


def backward(W, X, cache, dy):
    """Gradient of sum_b dy_b y_b with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(W)
    X = np.asarray(X, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    z1, h1, z2, h2 = cache
    dw3 = h2.T @ dy
    db3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def pinball(y, target, tau):
    """Mean pinball loss and its gradient with respect to y."""
    y = np.asarray(y, dtype=np.float64)
    r = np.asarray(target, dtype=np.float64) - y
    loss = np.where(r > 0, tau * r, (tau - 1.0) * r)
    dy = np.where(r > 0, -tau, np.where(r < 0, 1.0 - tau, 0.0)) / y.size
    return float(loss.mean()), dy


def adam(W, g, m1, m2, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1**t)
    vh = m2 / (1 - b2**t)
    return W - lr * mh / (np.sqrt(vh) + eps), m1, m2


def id_residual_at(A, X, J, k):
    """||A - A(:, J_k) Z_k||_F / ||A||_F with Z_k from the first k sketch rows."""
    Z = O.id_coeffs(X, J[:k], k)
    return O.residuals(A, J[:k], Z=Z, only=("id",))["id"]


def rank_label(A, Omega, tol, lmax):
    """Smallest k <= lmax with ID residual <= tol (scan of every k), or None."""
    A = np.asarray(A, dtype=np.float64)
    X = O.sketch(A, Omega)
    col = O.lupp_colwise(X, lmax)
    J = col["J"]
    for k in range(1, col["k_eff"] + 1):
        if id_residual_at(A, X, J, k) <= tol:
            return k
    return None
