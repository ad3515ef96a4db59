"""CPU oracle of the learned-setup surrogate network -- test infrastructure only.

Not part of the paper: the learned form replaces the local solves of the
harmonic extension (eq. (sparseP)) by a small network that maps a normalised
extension block D^{-1/2} A_BB D^{-1/2} to its inverse.  This module is the
plain FP64 reference of that network's arithmetic, used to check the GPU
kernels' forward and backward passes ("parity unpinned" by the paper: there is
nothing in the paper to pin it to; it is pinned by finite differences).

Network: features x (64) -> ReLU(x W1 + b1) (128) -> ReLU(. W2 + b2) (128)
-> . W3 + b3 (64).  Every matrix product takes its two operands rounded to
bfloat16 (round to nearest even) and accumulates exactly (FP64 here, FP32 on
the GPU); biases, activations and the loss are FP32/FP64.
"""
from __future__ import annotations

import numpy as np

F_IN, HID, F_OUT = 64, 128, 64
SMAX = 8


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest, ties to even); returns float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def packed_index(s=SMAX):
    """Row-major packed lower triangle (i, j), j <= i, of an s x s matrix."""
    return [(i, j) for i in range(s) for j in range(i + 1)]


def features_and_target(Abb):
    """Features and target of one extension block (size s <= 8):
    Ahat = D^{-1/2} A_BB D^{-1/2} padded with the identity to 8 x 8; features =
    its packed lower triangle (36) then log10 of the diagonal of A_BB minus
    their mean (s entries, zero padded) -> 64 values; target = packed lower
    triangle of Ahat^{-1} (36, zero padded to 64)."""
    s = Abb.shape[0]
    d = np.diag(Abb).astype(np.float64)
    Ah = Abb / np.sqrt(np.outer(d, d))
    M = np.eye(SMAX)
    M[:s, :s] = Ah
    W = np.eye(SMAX)
    W[:s, :s] = np.linalg.inv(Ah)
    idx = packed_index()
    x = np.zeros(F_IN)
    x[:36] = [M[i, j] for i, j in idx]
    ld = np.log10(d)
    x[36:36 + s] = ld - ld.mean()
    t = np.zeros(F_OUT)
    t[:36] = [W[i, j] for i, j in idx]
    return x, t


def _identity(a):
    return np.asarray(a, dtype=np.float64)


def forward(params, X, rounding=True):
    """Returns (Y, cache).  X: (N, 64) float array (already bf16-representable).
    rounding=False drops the bf16 rounding (plain FP64 network)."""
    rnd = bf16_round if rounding else _identity
    W1, b1, W2, b2, W3, b3 = params
    Xb = rnd(X)
    Z1 = Xb @ rnd(W1) + b1
    H1 = np.maximum(Z1, 0.0)
    H1b = rnd(H1)
    Z2 = H1b @ rnd(W2) + b2
    H2 = np.maximum(Z2, 0.0)
    H2b = rnd(H2)
    Y = H2b @ rnd(W3) + b3
    return Y, (Xb, Z1, H1b, Z2, H2b)


def backward(params, cache, dY, rounding=True):
    """Gradients of sum(dY * Y) with respect to every parameter, with the same
    bf16 rounding of matrix-product operands as the forward pass (the rounding
    itself is passed through unchanged, as a straight-through estimator)."""
    rnd = bf16_round if rounding else _identity
    W1, b1, W2, b2, W3, b3 = params
    Xb, Z1, H1b, Z2, H2b = cache
    dYb = rnd(dY)
    gW3 = H2b.T @ dYb
    gb3 = dY.sum(axis=0)
    dH2 = (dYb @ rnd(W3).T) * (Z2 > 0)
    dH2b = rnd(dH2)
    gW2 = H1b.T @ dH2b
    gb2 = dH2.sum(axis=0)
    dH1 = (dH2b @ rnd(W2).T) * (Z1 > 0)
    dH1b = rnd(dH1)
    gW1 = Xb.T @ dH1b
    gb1 = dH1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def unpack_sym(v, s=SMAX):
    """Symmetric s x s matrix from its packed lower triangle."""
    M = np.zeros((s, s))
    for q, (i, j) in enumerate(packed_index(s)):
        M[i, j] = M[j, i] = v[q]
    return M


def a_loss_grad(Y, T, Ahat, nvalid):
    """Training loss of the learned form: per row, the error of the predicted
    inverse W against the exact W* in the block's metric, ||Ahat (W - W*)||_F^2
    (equal to the refinement residual ||Ahat W - I||_F^2, as Ahat W* = I).
    Returns (row losses, gradient of their mean over the first nvalid rows with
    respect to Y); padding rows get zeros."""
    n = Y.shape[0]
    loss = np.zeros(n)
    G = np.zeros_like(Y, dtype=np.float64)
    idx = packed_index()
    for r in range(nvalid):
        A = unpack_sym(Ahat[r][:36])
        E = unpack_sym(np.asarray(Y[r][:36], float) - np.asarray(T[r][:36], float))
        AE = A @ E
        loss[r] = float((AE * AE).sum())
        Gm = 2.0 * A @ AE
        for q, (i, j) in enumerate(idx):
            G[r, q] = Gm[i, i] if i == j else Gm[i, j] + Gm[j, i]
    return loss, G / max(nvalid, 1)


def mse_grad(Y, T, mask):
    """Loss (1/N) sum mask * (Y - T)^2 and its gradient with respect to Y."""
    N = Y.shape[0]
    R = (Y - T) * mask
    return float((R * R).sum() / N), 2.0 * R / N
