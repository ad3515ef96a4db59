"""Pins of the learned-setup network's CPU oracle (oracle/mlp.py).

The network is an addition outside the paper, so nothing in the paper fixes
its values: the oracle is pinned by finite differences of its own forward pass
(without the bf16 rounding, which has no derivative), by torch's bfloat16
conversion, and by the algebra of the features and targets (the target is the
inverse of the normalised block, invariant under a scaling of the block).
"""
import numpy as np
import pytest
import torch

from gen.mlp_init import init_params, flatten, unflatten, N_PARAMS
from oracle import mlp


def test_bf16_round_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0]])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)
    # halfway cases go to the even neighbour
    assert mlp.bf16_round(np.float32(1.0 + 2 ** -8)) == 1.0
    assert mlp.bf16_round(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6


def _loss(params, X, T, mask):
    Y, _ = mlp.forward(params, X, rounding=False)
    return mlp.mse_grad(Y, T, mask)[0]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = init_params(3)
    params[1] = rng.standard_normal(mlp.HID) * 0.1
    params[3] = rng.standard_normal(mlp.HID) * 0.1
    params[5] = rng.standard_normal(mlp.F_OUT) * 0.1
    X = rng.standard_normal((6, mlp.F_IN))
    T = rng.standard_normal((6, mlp.F_OUT))
    mask = np.zeros((1, mlp.F_OUT))
    mask[0, :36] = 1.0
    Y, cache = mlp.forward(params, X, rounding=False)
    _, dY = mlp.mse_grad(Y, T, mask)
    grads = mlp.backward(params, cache, dY, rounding=False)
    h = 1e-6
    for k in range(6):
        flat = params[k].ravel()
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            pp = [p.copy() for p in params]
            pm = [p.copy() for p in params]
            pp[k].ravel()[idx] += h
            pm[k].ravel()[idx] -= h
            fd = (_loss(pp, X, T, mask) - _loss(pm, X, T, mask)) / (2 * h)
            an = grads[k].ravel()[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, idx, fd, an)


def test_mse_grad_matches_finite_differences():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((4, 64))
    T = rng.standard_normal((4, 64))
    mask = (rng.random((1, 64)) < 0.5).astype(float)
    L, g = mlp.mse_grad(Y, T, mask)
    assert L == pytest.approx(((Y - T) ** 2 * mask).sum() / 4)
    h = 1e-7
    for (i, j) in [(0, 0), (1, 5), (3, 63), (2, 17)]:
        Yp = Y.copy(); Yp[i, j] += h
        Ym = Y.copy(); Ym[i, j] -= h
        fd = (mlp.mse_grad(Yp, T, mask)[0] - mlp.mse_grad(Ym, T, mask)[0]) / (2 * h)
        assert fd == pytest.approx(g[i, j], abs=1e-7)


def _unpack(v, s=8):
    M = np.zeros((s, s))
    for q, (i, j) in enumerate(mlp.packed_index(s)):
        M[i, j] = M[j, i] = v[q]
    return M


@pytest.mark.parametrize("s", [1, 3, 6, 8])
def test_features_target_is_inverse_and_scale_invariant(s):
    rng = np.random.default_rng(10 + s)
    B = rng.standard_normal((s, s))
    A = B @ B.T + s * np.eye(s)
    D = np.diag(10.0 ** rng.uniform(-3, 3, s))
    A = D @ A @ D
    x, t = mlp.features_and_target(A)
    M = _unpack(x[:36])
    W = _unpack(t[:36])
    np.testing.assert_allclose(M @ W, np.eye(8), atol=1e-12)
    np.testing.assert_allclose(np.diag(M), 1.0)
    # padding is the identity; unused feature and target slots are zero
    np.testing.assert_array_equal(M[s:, s:], np.eye(8 - s))
    np.testing.assert_array_equal(M[:s, s:], 0.0)
    assert np.all(x[36 + s:] == 0.0) and np.all(t[36:] == 0.0)
    # the log10 diagonal features are centred
    assert abs(x[36:36 + s].sum()) < 1e-12
    # A_BB^{-1} = D^{-1/2} W D^{-1/2}
    d = np.sqrt(np.diag(A))
    np.testing.assert_allclose(W[:s, :s] / np.outer(d, d), np.linalg.inv(A), rtol=1e-9,
                               atol=1e-12 * np.abs(np.linalg.inv(A)).max())
    # a scaled block has the same features and target
    x2, t2 = mlp.features_and_target(7.5 * A)
    np.testing.assert_allclose(x2, x, atol=1e-12)
    np.testing.assert_allclose(t2, t, atol=1e-12)


def test_init_layout_roundtrip():
    p = init_params(0)
    f = flatten(p)
    assert f.size == N_PARAMS == 33088
    for a, b in zip(unflatten(f), p):
        np.testing.assert_array_equal(a, np.asarray(b, dtype=np.float32).astype(np.float64))


def _spd_packed(rng, s):
    B = rng.standard_normal((s, s))
    A = B @ B.T + s * np.eye(s)
    d = np.sqrt(np.diag(A))
    A = A / np.outer(d, d)
    M = np.eye(8)
    M[:s, :s] = A
    return np.array([M[i, j] for i, j in mlp.packed_index()]), M


def test_a_loss_equals_refinement_residual_and_gradient_is_exact():
    """||Ahat (W - W*)||^2 = ||Ahat W - I||^2 when W* = Ahat^{-1}; the gradient
    matches central differences of the loss in the packed outputs."""
    rng = np.random.default_rng(7)
    n, nvalid = 5, 4
    Ah = np.zeros((n, 36))
    Y = np.zeros((n, 64))
    T = np.zeros((n, 64))
    for r in range(n):
        Ah[r], M = _spd_packed(rng, int(rng.integers(1, 9)))
        Winv = np.linalg.inv(M)
        T[r, :36] = [Winv[i, j] for i, j in mlp.packed_index()]
        Y[r, :36] = T[r, :36] + 0.1 * rng.standard_normal(36)
        Y[r, 36:] = rng.standard_normal(28)     # unused outputs: no loss, no gradient
    loss, G = mlp.a_loss_grad(Y, T, Ah, nvalid)
    for r in range(nvalid):
        W = mlp.unpack_sym(Y[r, :36])
        R = mlp.unpack_sym(Ah[r]) @ W - np.eye(8)
        assert loss[r] == pytest.approx((R * R).sum(), rel=1e-10)
    assert loss[nvalid] == 0.0 and np.all(G[nvalid] == 0.0) and np.all(G[:, 36:] == 0.0)
    h = 1e-6
    mean = lambda YY: mlp.a_loss_grad(YY, T, Ah, nvalid)[0].sum() / nvalid
    for r, q in [(0, 0), (0, 5), (1, 20), (2, 35), (3, 14)]:
        Yp = Y.copy(); Yp[r, q] += h
        Ym = Y.copy(); Ym[r, q] -= h
        assert (mean(Yp) - mean(Ym)) / (2 * h) == pytest.approx(G[r, q], rel=1e-6, abs=1e-9)
