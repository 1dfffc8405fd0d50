"""Learned rank selection on top of the randomized LUPP path (added form,
not in the paper).

A small MLP (512 -> 128 -> 128 -> 1, FP32) reads the pivot-magnitude
profile |u_tt| of the FP32 LUPP of a BF16 sketch (the pivots of eq.
(def_LUPP) computed by Alg. 2 step 3 over all l steps) and predicts log2 of
the smallest rank k whose interpolative decomposition (Sec. 4) meets a
relative Frobenius tolerance.  Labels come from the plain FP64 path on the
GPU; the plain path with rank doubling is both the fallback and the reference.

Every arithmetic step runs in the library's kernels through the C-ABI
(sketch, LUPP, features, forward, loss, backward, Adam, Z, residual); this
module only sequences the calls and moves small index/feature tensors.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import rpid as R

FEAT = R.MLP_IN  # 512 profile entries
RANK_CAP = 1024  # largest rank the library's LUPP, Z and residual accept


# ---------------------------------------------------------------------------
# features and labels
# ---------------------------------------------------------------------------
def profile(ctx, A_lo, Om_lo, l):
    """Sketch X = Omega A in the storage type of A_lo (BF16 gives an FP32
    sketch) and its LUPP over all l steps: (features, |u_tt| on the device,
    k_eff); the features are f_t = max(log10(|u_tt| / |u_00|), -20) (FEAT
    entries, -20 beyond k_eff)."""
    X = R.rpid_sketch(ctx, A_lo, Om_lo[:l])
    J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, X, l)
    return R.rpid_mlp_features(ctx, diag, FEAT, keff), diag, keff


def profile_features(ctx, A_lo, Om_lo, l):
    """The network's input for one matrix (see profile)."""
    return profile(ctx, A_lo, Om_lo, l)[0]


class PlainPath:
    """The plain FP64 path at any rank k <= lmax for one matrix: one FP64
    sketch of lmax rows and one LUPP of lmax steps serve every k (the first k
    pivots and factors depend only on the first k sketch rows)."""

    def __init__(self, ctx, A64, Om64, lmax):
        self.ctx, self.A = ctx, A64
        self.X = R.rpid_sketch(ctx, A64, Om64[:lmax])
        self.J, self.Lf, self.Uf, _, self.k_eff, _ = R.rpid_select_columns(ctx, self.X, lmax)
        self.evals = 0

    def residual(self, k):
        Z, _ = R.rpid_id_coeffs(self.ctx, self.X, k, self.J, self.Lf, self.Uf, refine_steps=0)
        self.evals += 1
        return R.rpid_residual(self.ctx, R.RESIDUAL_ID, self.A, k, self.J, Z=Z)


def rank_label(ctx, A64, Om64, tol, lmax):
    """Smallest k <= lmax whose ID residual is <= tol, by bisection over the
    ranks (the residual is taken as non-increasing in k; the result always
    satisfies residual(k) <= tol < residual(k - 1)).  None if rank lmax fails.
    Returns (label, number of residual evaluations)."""
    p = PlainPath(ctx, A64, Om64, lmax)
    hi = p.k_eff
    if hi < 1 or p.residual(hi) > tol:
        return None, p.evals
    lo = 0  # residual(lo) > tol (rank 0: the whole matrix)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if p.residual(mid) <= tol:
            hi = mid
        else:
            lo = mid
    return hi, p.evals


def target_of(label, lmax):
    """log2 k*; a censored matrix (no k <= lmax) gets log2(lmax + 1)."""
    return math.log2(label if label is not None else lmax + 1)


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------
class RankNet:
    """MLP weights and Adam state on the device; training and inference run in
    the library's kernels."""

    def __init__(self, ctx, seed=0, device="cuda"):
        self.ctx = ctx
        rng = np.random.default_rng([seed, 77])
        parts = []
        for fan_in, fan_out in ((R.MLP_IN, R.MLP_H), (R.MLP_H, R.MLP_H), (R.MLP_H, 1)):
            a = math.sqrt(6.0 / (fan_in + fan_out))  # Xavier-uniform
            parts.append(rng.uniform(-a, a, fan_in * fan_out))
            parts.append(np.zeros(fan_out))
        w = np.concatenate(parts).astype(np.float32)
        assert w.size == R.MLP_NPARAM
        self.W = torch.from_numpy(w).to(device)
        self.m1 = torch.zeros_like(self.W)
        self.m2 = torch.zeros_like(self.W)
        self.t = 0

    def predict(self, feats):
        y, _ = R.rpid_mlp_forward(self.ctx, self.W, feats, want_act=False)
        return y

    def step(self, feats, targets, tau, lr):
        """One Adam step on a batch; returns the batch loss (device tensor)."""
        y, act = R.rpid_mlp_forward(self.ctx, self.W, feats, want_act=True)
        loss, dy = R.rpid_mlp_loss(self.ctx, y, targets, tau)
        dW = R.rpid_mlp_backward(self.ctx, self.W, feats, act, dy)
        self.t += 1
        R.rpid_mlp_adam(self.ctx, self.W, dW, self.m1, self.m2, lr, self.t)
        return loss

    def fit(self, feats, targets, epochs=200, batch=64, lr=1e-3, tau=0.9, seed=0):
        """Mini-batch Adam over (feats N x 512, targets N); returns the mean
        loss of each epoch (host floats)."""
        N = feats.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        hist = []
        for _ in range(epochs):
            perm = torch.randperm(N, generator=g).to(feats.device)
            losses = []
            for s in range(0, N, batch):
                idx = perm[s:s + batch]
                losses.append(self.step(feats[idx].contiguous(), targets[idx].contiguous(), tau, lr))
            hist.append(float(torch.stack(losses).mean()))
        return hist


# ---------------------------------------------------------------------------
# reaching a tolerance
# ---------------------------------------------------------------------------
def attempt(ctx, A64, Om64, k):
    """The plain FP64 path at rank k: sketch with the first k rows of Omega,
    k LUPP steps, Z, and the relative ID residual."""
    X = R.rpid_sketch(ctx, A64, Om64[:k])
    J, Lf, Uf, _, k_eff, st = R.rpid_select_columns(ctx, X, k)
    if st != 0:
        # an exactly zero pivot: the sketch has rank k_eff; evaluate rank k_eff
        if k_eff < 1:
            return 1.0
        k = k_eff
    Z, _ = R.rpid_id_coeffs(ctx, X, k, J, Lf, Uf, refine_steps=0)
    return R.rpid_residual(ctx, R.RESIDUAL_ID, A64, k, J, Z=Z)


def _double_until(ctx, A64, Om64, tol, k, lmax):
    evals = 0
    while True:
        evals += 1
        if attempt(ctx, A64, Om64, k) <= tol:
            return k, evals
        if k >= lmax:
            return None, evals
        k = min(2 * k, lmax)


def solve_doubling(ctx, A64, Om64, tol, k0, lmax):
    """Plain FP64 path with rank doubling from k0: (k, attempts, seconds);
    k = None when rank lmax does not meet tol."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k, evals = _double_until(ctx, A64, Om64, tol, min(k0, lmax), lmax)
    torch.cuda.synchronize()
    return k, evals, time.perf_counter() - t0


def rank_of(y, shift, lmax):
    """k_hat = ceil(2^(y + shift)) clamped to [1, lmax]."""
    return int(min(max(math.ceil(2.0 ** (float(y) + shift)), 1), lmax))


def predict_rank(ctx, net, A_lo, Om_lo, l_feat, lmax, shift=0.0):
    """k_hat from the profile of a low-precision sketch (clamped to [1, lmax])."""
    f = profile_features(ctx, A_lo, Om_lo, l_feat)
    return rank_of(net.predict(f.view(1, FEAT))[0], shift, lmax)


def solve_learned(ctx, net, A64, Om64, A_lo, Om_lo, tol, l_feat, lmax, shift=0.0):
    """Profile of the BF16 sketch's FP32 LUPP -> network -> k_hat, then the
    plain FP64 path from k_hat with rank doubling as the fallback (up to
    lmax, which may exceed l_feat): (k, attempts, seconds, k_hat)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k_hat = predict_rank(ctx, net, A_lo, Om_lo, l_feat, lmax, shift)
    k, evals = _double_until(ctx, A64, Om64, tol, k_hat, lmax)
    torch.cuda.synchronize()
    return k, evals, time.perf_counter() - t0, k_hat


def solve_threshold(ctx, A64, Om64, A_lo, Om_lo, tol, l_feat, lmax):
    """Non-learned comparison: the same profile, k from the pivot-ratio rule
    (threshold_rank), then the plain FP64 path with rank doubling:
    (k, attempts, seconds, k_rule)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, diag, keff = profile(ctx, A_lo, Om_lo, l_feat)
    k_rule = threshold_rank(diag[:max(keff, 1)].double().cpu().tolist(), tol)
    k, evals = _double_until(ctx, A64, Om64, tol, min(k_rule, lmax), lmax)
    torch.cuda.synchronize()
    return k, evals, time.perf_counter() - t0, k_rule


def modelled_cost(k_start, label, lmax, c0=32.0):
    """Cost, in rank units, of reaching the tolerance from k_start with rank
    doubling: an attempt at rank k costs k + c0 (sketch, LUPP steps and
    residual all grow with k); a censored label (None) runs up to lmax."""
    target = lmax if label is None else label
    k, cost = k_start, 0.0
    while True:
        cost += k + c0
        if k >= target or k >= lmax:
            return cost
        k = min(2 * k, lmax)


def calibrate_shift(y_pred, labels, lmax, grid=None):
    """The shift (log2 units) added to the network's outputs that minimises
    the summed modelled cost over a calibration set the network was not
    fitted on (a miss costs a doubling, an overshoot costs rank)."""
    if grid is None:
        grid = np.arange(-1.0, 2.0001, 0.05)
    best = None
    for d in grid:
        c = sum(modelled_cost(rank_of(y, d, lmax), lab, lmax) for y, lab in zip(y_pred, labels))
        if best is None or c < best[0]:
            best = (c, float(d))
    return best[1]


def threshold_rank(diag, tol):
    """Non-learned rule for comparison: the first t with |u_tt| / |u_00| < tol
    (host list of pivot magnitudes), or len(diag) if none."""
    d0 = float(diag[0])
    for t, d in enumerate(diag):
        if float(d) < tol * d0:
            return max(t, 1)
    return len(diag)
