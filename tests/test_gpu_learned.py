"""GPU checks of the learned-setup form (an addition outside the paper).

The network's kernels are checked against the CPU oracle (oracle/mlp.py):
bit-exactly on inputs whose every partial sum is exact in FP32 (so that both
sides round every bf16 operand the same way), and norm-wise on realistic
inputs.  The learned finest-level interpolation is checked against the
oracle's exact P (eq. (sparseP)) with a bound derived from the acceptance
test, and the solver built on it against the oracle's PCG iteration count.
Every call goes through the C ABI.
"""
import numpy as np
import pytest

from gen.mlp_init import init_params, flatten, unflatten, N_PARAMS
from oracle import mlp as omlp
from test_gpu_parity import case, dev, _rowwise_err, EPS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle                             # noqa: E402
import paper_2602_23613_amd as amglib     # noqa: E402


def _bf16(X):
    """Device bf16 tensor of values that are already bf16-representable."""
    t = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(torch.bfloat16)
    assert np.array_equal(t.to(torch.float64).numpy(), np.asarray(X, dtype=np.float64))
    return t.to(dev())


def _gpu_pass(H, X, dY):
    d = dev()
    xb = _bf16(X)
    y = torch.zeros((X.shape[0], 64), dtype=torch.float32, device=d)
    H.mlp_forward(xb, y)
    g = torch.zeros(N_PARAMS, dtype=torch.float32, device=d)
    H.mlp_backward(xb, torch.tensor(dY, dtype=torch.float32, device=d), g)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), unflatten(g.cpu().numpy())


def _hier():
    p, _ = case("hex8_iso")
    return amglib.Hierarchy(p.A, p.G)


def _grid(rng, shape, lo, hi, denom):
    return rng.integers(lo, hi + 1, shape) / denom


@pytest.mark.parametrize("n", [16, 80])
def test_mlp_passes_bit_exact_on_exact_grid(n):
    """Operands on dyadic grids with bounded magnitude: every product and
    partial sum is exact in FP32 and FP64, so the GPU (MFMA, any summation
    order) and the oracle must agree bit for bit, which pins the MFMA operand
    layout, the transposes of the backward pass, the masks and the biases."""
    dev()
    rng = np.random.default_rng(100 + n)
    params = [_grid(rng, (64, 128), -4, 4, 16), _grid(rng, 128, -16, 16, 256),
              _grid(rng, (128, 128), -4, 4, 16), _grid(rng, 128, -64, 64, 4096),
              _grid(rng, (128, 64), -4, 4, 16), _grid(rng, 64, -64, 64, 65536)]
    X = _grid(rng, (n, 64), -4, 4, 16)
    dY = _grid(rng, (n, 64), -2, 2, 8)
    Y, cache = omlp.forward(params, X)
    grads = omlp.backward(params, cache, dY)
    Xb, Z1, H1b, Z2, H2b = cache
    # exactness preconditions: sum |a||b| < 2^24 * grid for every contraction
    W = [omlp.bf16_round(w) for w in params[0::2]]
    assert (np.abs(Xb) @ np.abs(W[0])).max() < 2.0 ** 24 * 2.0 ** -8
    assert (np.abs(H1b) @ np.abs(W[1])).max() < 2.0 ** 24 * 2.0 ** -12
    assert (np.abs(H2b) @ np.abs(W[2])).max() < 2.0 ** 24 * 2.0 ** -16
    assert (np.abs(H2b).T @ np.abs(dY)).max() < 2.0 ** 24 * 2.0 ** -15
    H = _hier()
    H.mlp_params(set=flatten(params))
    Yg, gg = _gpu_pass(H, X, dY)
    np.testing.assert_array_equal(Yg, Y)
    for k in range(6):
        np.testing.assert_array_equal(gg[k], grads[k], err_msg=f"parameter block {k}")
    H.close()


def _block_features(p, H, limit=None):
    """Oracle features of the library's finest-level extension blocks."""
    ints = H.integers(0)
    bp, bd = np.asarray(ints["block_ptr"]), np.asarray(ints["block_dofs"])
    A = p.A.tocsr()
    X, T = [], []
    for b in range(len(bp) - 1 if limit is None else min(limit, len(bp) - 1)):
        dofs = bd[bp[b]:bp[b + 1]]
        x, t = omlp.features_and_target(A[dofs][:, dofs].toarray())
        X.append(x)
        T.append(t)
    return np.array(X), np.array(T)


def test_mlp_passes_on_block_features():
    """Realistic inputs (features of hex12 extension blocks, random weights):
    the GPU accumulates in FP32, so a bf16 rounding of an activation may land
    on the other side of a tie; each such flip moves one term by one bf16 ulp
    (2^-8 relative), so the outputs agree norm-wise to ~2^-8."""
    dev()
    p, _ = case("hex12_jump")
    H = amglib.Hierarchy(p.A, p.G)
    X, _ = _block_features(p, H, limit=256)
    X = omlp.bf16_round(X)
    rng = np.random.default_rng(5)
    params = init_params(1)
    for k in (1, 3, 5):
        params[k] = rng.standard_normal(params[k].shape) * 0.1
    params = unflatten(flatten(params))
    dY = rng.standard_normal(X.shape[:1] + (64,)) / X.shape[0]
    Y, cache = omlp.forward(params, X)
    grads = omlp.backward(params, cache, dY)
    H.mlp_params(set=flatten(params))
    Yg, gg = _gpu_pass(H, X, dY)
    ey = np.linalg.norm(Yg - Y) / np.linalg.norm(Y)
    print(f"forward rel err {ey:.2e}")
    assert ey <= 2.0 ** -8
    for k in range(6):
        eg = np.linalg.norm(gg[k] - grads[k]) / np.linalg.norm(grads[k])
        print(f"grad {k} rel err {eg:.2e}")
        assert eg <= 2.0 ** -6, k
    H.close()


def _learned_bound(p, H, tol):
    """Relative error bound of a learned block solve accepted with
    ||Ahat W - I||_F <= tol: X_B - X_B* = A_BB^{-1} D^{1/2} E D^{-1/2} R_B with
    ||E|| <= tol, so the relative error is at most kappa(A_BB) sqrt(kappa(D))
    tol; one later stage can pass it on once more (factor 2), and exact
    rounding adds the 8 kappa eps of the exact path."""
    ints = H.integers(0)
    bp, bd = np.asarray(ints["block_ptr"]), np.asarray(ints["block_dofs"])
    A = p.A.tocsr()
    worst, kmax = 0.0, 1.0
    for b in range(len(bp) - 1):
        dofs = bd[bp[b]:bp[b + 1]]
        Abb = A[dofs][:, dofs].toarray()
        d = np.diag(Abb)
        k = np.linalg.cond(Abb)
        kmax = max(kmax, k)
        worst = max(worst, k * np.sqrt(d.max() / d.min()))
    return 2 * worst * tol + 8 * kmax * EPS


# (case, required loss reduction, required accepted fraction of the trained-on blocks)
LEARN_CASES = [("hex8_iso", 0.05, 0.95), ("hex12_jump", 0.5, 0.9)]


@pytest.mark.parametrize("name,loss_ratio,acc_frac", LEARN_CASES)
def test_learned_setup_matches_exact(name, loss_ratio, acc_frac):
    d = dev()
    p, Ho = case(name)
    H = amglib.Hierarchy(p.A, p.G)
    st = H.mlp_train(epochs=300, batch=64, lr=2e-3, seed=1, init=flatten(init_params(0)),
                     global_iters=12)
    print("train", st)
    # eligibility: at most 8 DoFs and every entry of the normalised inverse <= 50
    _, T = _block_features(p, H)
    assert st["blocks"] == T.shape[0] > 0
    assert st["eligible"] == int((np.abs(T).max(axis=1) <= 50.0).sum())
    assert st["loss_last"] < loss_ratio * st["loss_first"]
    tol = 1e-10
    H.mlp_use(refine_steps=6, accept_tol=tol, global_iters=12, global_slack=0.02)
    H.resetup(p.A)
    su = H.mlp_stats()
    print("use", su)
    assert su["global_fallback"] == 0
    assert su["accepted"] > 0 and su["accepted"] >= acc_frac * st["eligible"]
    assert su["rho_learned"] <= su["rho_reference"] + 0.02
    _, P0 = H.level(0)
    eP = _rowwise_err(P0, Ho.levels[0].P)
    bound = _learned_bound(p, H, tol)
    print(f"learned P rel err {eP:.2e} (bound {bound:.1e})")
    assert eP <= bound
    f = torch.tensor(p.f, device=d)
    u = torch.zeros_like(f)
    s = H.pcg(f, u, rtol=1e-8, maxit=500)
    _, it_o, _ = oracle.pcg(Ho, p.A, p.f, maxit=500)
    tol_its = 1 if s["replacements"] == 0 else max(3, 0.1 * it_o)
    assert s["status"] == 0 and abs(s["iterations"] - it_o) <= tol_its, (s["iterations"], it_o)
    uu = u.cpu().numpy()
    assert np.linalg.norm(p.f - p.A @ uu) / np.linalg.norm(p.f) <= 2e-8
    H.close()


def test_rejected_predictions_fall_back_to_exact_bitwise():
    """An all-zero network predicts W = 0, so ||Ahat W - I|| = sqrt(s) >= 1:
    every block is rejected and the setup must equal the exact one bit for
    bit.  The same holds when the global check is forced to fail (negative
    slack): the whole numeric setup is redone exactly."""
    d = dev()
    p, _ = case("hex8_iso")
    H = amglib.Hierarchy(p.A, p.G)
    _, P_exact = H.level(0)
    r = torch.tensor(np.random.default_rng(9).standard_normal(p.A.shape[0]), device=d)
    z0 = torch.zeros_like(r)
    H.vcycle(r, z0)
    H.mlp_params(set=np.zeros(N_PARAMS, np.float32))
    H.mlp_use(refine_steps=4, accept_tol=1e-10)
    H.resetup(p.A)
    assert H.mlp_stats()["accepted"] == 0
    _, P1 = H.level(0)
    assert np.array_equal(P1.data, P_exact.data)
    z1 = torch.zeros_like(r)
    H.vcycle(r, z1)
    torch.cuda.synchronize()
    assert torch.equal(z0, z1)
    # a trained network with a global check that cannot pass
    H.mlp_train(epochs=200, batch=64, lr=2e-3, seed=2, init=flatten(init_params(0)),
                global_iters=8)
    H.mlp_use(refine_steps=6, accept_tol=1e-10, global_iters=8, global_slack=-10.0)
    H.resetup(p.A)
    s = H.mlp_stats()
    assert s["global_fallback"] == 1 and s["accepted"] == 0
    _, P2 = H.level(0)
    assert np.array_equal(P2.data, P_exact.data)
    z2 = torch.zeros_like(r)
    H.vcycle(r, z2)
    torch.cuda.synchronize()
    assert torch.equal(z0, z2)
    # disabling the learned form restores the exact setup as well
    H.mlp_use(enable=False)
    H.resetup(p.A)
    _, P3 = H.level(0)
    assert np.array_equal(P3.data, P_exact.data)
    H.close()


def test_learned_api_errors():
    dev()
    H = _hier()
    with pytest.raises(amglib.AmgError):
        H.mlp_use()                          # no parameters yet
    with pytest.raises(amglib.AmgError):
        H.mlp_train(epochs=1, batch=64)      # first training needs init
    with pytest.raises(amglib.AmgError):
        H.mlp_train(epochs=1, batch=24, init=flatten(init_params(0)))   # batch not a multiple of 16
    H.close()


def test_training_loss_kernel_matches_oracle():
    """The training loss ||Ahat (W - W*)||^2 and its gradient, GPU against the
    oracle (both evaluate in FP64; the GPU rounds the results to FP32)."""
    d = dev()
    rng = np.random.default_rng(31)
    n, nvalid = 40, 33
    Ah = np.zeros((n, 36))
    T = np.zeros((n, 64), np.float32)
    Y = np.zeros((n, 64), np.float32)
    idx = omlp.packed_index()
    for r in range(n):
        s = int(rng.integers(1, 9))
        B = rng.standard_normal((s, s))
        A = B @ B.T + s * np.eye(s)
        dd = np.sqrt(np.diag(A))
        M = np.eye(8)
        M[:s, :s] = A / np.outer(dd, dd)
        Ah[r] = [M[i, j] for i, j in idx]
        W = np.linalg.inv(M)
        T[r, :36] = [W[i, j] for i, j in idx]
        Y[r, :36] = T[r, :36] + 0.05 * rng.standard_normal(36)
        Y[r, 36:] = rng.standard_normal(28)
    loss_o, G_o = omlp.a_loss_grad(Y.astype(np.float64), T.astype(np.float64), Ah, nvalid)
    yt = torch.tensor(Y, device=d)
    tt = torch.tensor(T, device=d)
    at = torch.tensor(Ah, device=d)
    dy = torch.full((n, 64), 7.0, dtype=torch.float32, device=d)
    rl = torch.full((n,), 7.0, dtype=torch.float32, device=d)
    amglib.mlp_loss_grad(yt, tt, at, nvalid, dy, rl)
    torch.cuda.synchronize()
    np.testing.assert_allclose(rl.cpu().numpy(), loss_o, rtol=2e-7, atol=1e-30)
    g = dy.cpu().numpy().astype(np.float64)
    scale = np.abs(G_o).max(axis=1, keepdims=True) + 1e-30
    assert np.max(np.abs(g - G_o) / scale) <= 2e-7
    assert np.all(g[nvalid:] == 0.0) and np.all(g[:, 36:] == 0.0)


def test_chunked_inference_equals_one_pass():
    """Inference runs in passes of at most 16384 rows; forcing passes of 32
    rows must give the same accepted blocks and the same P bit for bit."""
    import os
    dev()
    p, _ = case("hex8_iso")
    H = amglib.Hierarchy(p.A, p.G)
    H.mlp_train(epochs=200, batch=64, lr=2e-3, seed=3, init=flatten(init_params(0)))
    H.mlp_use(refine_steps=6, accept_tol=1e-10)
    H.resetup(p.A)
    a1 = H.mlp_stats()["accepted"]
    _, P1 = H.level(0)
    os.environ["HCURL_AMG_INFER_ROWS"] = "32"
    try:
        H.resetup(p.A)
    finally:
        del os.environ["HCURL_AMG_INFER_ROWS"]
    assert H.mlp_stats()["accepted"] == a1 > 0
    _, P2 = H.level(0)
    assert np.array_equal(P1.data, P2.data)
    H.close()


def test_learned_setup_on_a_new_field():
    """The use the learned form is for: train on the exact local solves of one
    coefficient field, then re-set up on another field of the same law.  The
    accepted blocks must reproduce the exact P of the new field within the
    acceptance bound, and most blocks must be accepted."""
    from gen import fields
    import gen
    import oracle as _or
    dev()
    law = lambda seed: (lambda m: fields.subdomain_log_uniform(m, 8, seed))
    p1 = gen.make_problem("hex", 16, beta=1.0, alpha=law(2))
    p2 = gen.make_problem("hex", 16, beta=1.0, alpha=law(12))
    H = amglib.Hierarchy(p1.A, p1.G)
    st = H.mlp_train(epochs=60, batch=256, lr=1e-3, seed=0, init=flatten(init_params(0)))
    print("train", {k: st[k] for k in ("blocks", "eligible", "loss_first", "loss_last")})
    H.mlp_use(refine_steps=6, accept_tol=1e-10)
    H.resetup(p2.A)
    su = H.mlp_stats()
    print("use", {k: su[k] for k in ("blocks", "eligible", "accepted")})
    Ho = _or.setup(p2.A, p2.G, max_levels=2)
    _, P0 = H.level(0)
    eP = _rowwise_err(P0, Ho.levels[0].P)
    bound = _learned_bound(p2, H, 1e-10)
    print(f"learned P rel err {eP:.2e} (bound {bound:.1e})")
    assert eP <= bound
    assert su["accepted"] >= 0.5 * st["eligible"]
    H.close()
