"""Parity at the full sizes of the hex workloads (64^3 and 128^3), on outputs the oracle's definitions give one by one and
on properties that hold at any size, in the launch configuration bench.py
times (device-resident A and G, FP64 hierarchy).

* local harmonic extension (eq. (sparseP)): sampled blocks of every stage of
  level 0 are recomputed densely from A and the GPU's own rows of the
  already-extended DoFs, X_B = -A_BB^{-1} A_{B,done} P_done, and compared with
  the GPU's rows to 8 kappa(A_BB) eps; exterior rows must equal R^T exactly;
* Galerkin entries of level 1, (P^T A P)_ij, recomputed from the GPU's P and
  A, to 64 eps (|P_i|^T |A| |P_j|) (a bound on the summation error);
* the V(1,1) cycle is symmetric and positive (exact in exact arithmetic);
* PCG's recursive residual agrees with the true residual.

At 64^3 the level-0 SpMV-with-dot of PCG runs 23,814 workgroups, more than
the fixed 2,048-slot grid of the other reductions: its partial-sum buffer
must be sized from its own grid (an earlier sizing from the smallest grid
overflowed it by 95 KB per iteration, corrupting later allocations).
"""
import os

import numpy as np
import pytest

import gen
from gen import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2602_23613_amd as amglib   # noqa: E402

EPS = np.finfo(np.float64).eps


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _workload(N):
    seed_a, seed_f = (2, 102) if N <= 64 else (3, 103)
    return gen.make_problem("hex", N, beta=1.0,
                            alpha=lambda m: fields.subdomain_log_uniform(m, 8, seed_a),
                            f=lambda n: fields.rhs_uniform(n, seed_f))


def _device_csr(M, d):
    return (torch.from_numpy(M.indptr.astype(np.int64)).to(d),
            torch.from_numpy(M.indices.astype(np.int32)).to(d),
            torch.from_numpy(M.data.astype(np.float64)).to(d), M.shape[0], M.shape[1])


def _check_extension(A, P, ints, rng, nsample=48):
    A = A.tocsr()
    P = P.tocsr()
    n = A.shape[0]
    bp = np.asarray(ints["block_ptr"])
    bd = np.asarray(ints["block_dofs"])
    depth = np.asarray(ints["block_depth"])
    dof_depth = np.full(n, -1, dtype=np.int64)      # -1: exterior (rows of R^T)
    for b in range(len(bp) - 1):
        dof_depth[bd[bp[b]:bp[b + 1]]] = depth[b]
    # exterior rows: exactly R^T (one +-1 per row, in the column of its coarse edge)
    nc = int(ints["nc"])
    for arr_d, arr_s in (("r_dof1", "r_s1"), ("r_dof2", "r_s2")):
        dd = np.asarray(ints[arr_d])
        ss = np.asarray(ints[arr_s])
        for c in rng.choice(nc, size=min(200, nc), replace=False):
            row = P[dd[c]]
            assert row.nnz == 1 and row.indices[0] == c and row.data[0] == ss[c]
    worst = 0.0
    for dep in np.unique(depth):
        ids = np.nonzero(depth == dep)[0]
        for b in rng.choice(ids, size=min(nsample, len(ids)), replace=False):
            B = bd[bp[b]:bp[b + 1]]
            AB = A[B]
            cols = np.unique(AB.indices)
            done = cols[(dof_depth[cols] < dep) & ~np.isin(cols, B)]
            pat = P[B[0]].indices
            rhs = (AB[:, done] @ P[done]).toarray()[:, pat]
            Abb = A[B][:, B].toarray()
            X = -np.linalg.solve(Abb, rhs)
            G = P[B].toarray()[:, pat]
            scale = np.maximum(np.abs(X).max(axis=1, keepdims=True), 1e-300)
            err = (np.abs(G - X) / scale).max()
            tol = max(1e-13, 8 * np.linalg.cond(Abb) * EPS)
            assert err <= tol, (int(b), int(dep), err, tol)
            worst = max(worst, err / tol)
    return worst


def _check_patch_extension(A, P, ints, rng, nsample=64):
    """Patch form: column c of P is R^T e_c on its two exterior DoFs and
    X_c = -A_SS^{-1} A_S,ext (R^T e_c) on its patch S (recomputed densely)."""
    A = A.tocsr()
    Pc = P.tocsc()
    pp = np.asarray(ints["patch_ptr"])
    pd = np.asarray(ints["patch_dofs"])
    d1, d2 = np.asarray(ints["r_dof1"]), np.asarray(ints["r_dof2"])
    s1, s2 = np.asarray(ints["r_s1"]), np.asarray(ints["r_s2"])
    nc = int(ints["nc"])
    worst = 0.0
    for c in rng.choice(nc, size=min(nsample, nc), replace=False):
        col = Pc[:, c]
        got = dict(zip(col.indices.tolist(), col.data.tolist()))
        assert got[int(d1[c])] == s1[c] and got[int(d2[c])] == s2[c]
        S = pd[pp[c]:pp[c + 1]]
        assert set(got) == set(S.tolist()) | {int(d1[c]), int(d2[c])}
        if len(S) == 0:
            continue
        rhs = A[S][:, [int(d1[c]), int(d2[c])]].toarray() @ np.array([s1[c], s2[c]], dtype=np.float64)
        Ass = A[S][:, S].toarray()
        X = -np.linalg.solve(Ass, rhs)
        G = np.array([got[int(j)] for j in S])
        err = np.abs(G - X).max() / max(np.abs(X).max(), 1e-300)
        tol = max(1e-13, 8 * np.linalg.cond(Ass) * EPS)
        assert err <= tol, (int(c), err, tol)
        worst = max(worst, err / tol)
    return worst


def _check_galerkin(A, P, A1, rng, nsample=300):
    Pc = P.tocsc()
    absA = abs(A)
    A1 = A1.tocsr()
    rows = np.repeat(np.arange(A1.shape[0]), np.diff(A1.indptr))
    pick = rng.choice(A1.nnz, size=min(nsample, A1.nnz), replace=False)
    worst = 0.0
    for q in pick:
        i, j = rows[q], A1.indices[q]
        pi, pj = Pc[:, i], Pc[:, j]
        v = (pi.T @ (A @ pj)).toarray()[0, 0]
        bound = 64 * EPS * (abs(pi).T @ (absA @ abs(pj))).toarray()[0, 0]
        e = abs(A1.data[q] - v)
        assert e <= bound, (int(i), int(j), e, bound)
        worst = max(worst, e / bound)
    return worst


def _fullsize(N, ext_mode="blocks"):
    d = dev()
    rng = np.random.default_rng(N)
    p = _workload(N)
    print(f"hex {N}^3, {ext_mode} extension", flush=True)
    H = amglib.Hierarchy(_device_csr(p.A, d), _device_csr(p.G, d), ext_mode=ext_mode)
    info = H.info()
    print("levels", [(l["n"], l["nnz"]) for l in info])
    A0, P0 = H.level(0)
    assert (A0 != p.A).nnz == 0
    ints = H.integers(0)
    if ext_mode == "patch":
        we = _check_patch_extension(A0, P0, ints, rng)
    else:
        we = _check_extension(A0, P0, ints, rng)
    A1, _ = H.level(1)
    wg = _check_galerkin(A0, P0, A1, rng)
    print(f"extension worst err/tol {we:.2e}; Galerkin worst err/bound {wg:.2e}")
    # V-cycle: symmetric and positive
    n = p.A.shape[0]
    r = torch.tensor(rng.standard_normal(n), device=d)
    s = torch.tensor(rng.standard_normal(n), device=d)
    zr, zs = torch.zeros_like(r), torch.zeros_like(r)
    H.vcycle(r, zr)
    H.vcycle(s, zs)
    torch.cuda.synchronize()
    a = torch.dot(s, zr).item()
    b = torch.dot(r, zs).item()
    scale = torch.linalg.norm(s).item() * torch.linalg.norm(zr).item()
    print(f"V-cycle symmetry |s.Br - r.Bs| / (|s||Br|) = {abs(a - b) / scale:.2e}")
    assert abs(a - b) <= 1e-8 * scale
    assert torch.dot(r, zr).item() > 0 and torch.dot(s, zs).item() > 0
    # PCG: recursive and true residual agree
    f = torch.tensor(p.f, device=d)
    u = torch.zeros_like(f)
    st = H.pcg(f, u, rtol=1e-8, maxit=60)
    uu = u.cpu().numpy()
    floor = 64 * EPS * np.linalg.norm(abs(p.A) @ np.abs(uu)) / np.linalg.norm(p.f)
    true = np.linalg.norm(p.f - p.A @ uu) / np.linalg.norm(p.f)
    print(f"PCG 60 its: recursive {st['relres']:.3e} true {true:.3e} (library {st['true_relres']:.3e})")
    assert st["relres"] < 1.0
    assert abs(true - st["true_relres"]) <= max(1e-6 * true, floor)
    assert abs(true - st["relres"]) <= 1e-3 * true + 1e3 * floor
    H.close()


def test_full_size_64():
    _fullsize(64)


def test_full_size_128():
    _fullsize(128)


def test_full_size_128_patch():
    """The 128^3 workload in the configuration of the bench.py headline
    (patch extension, device-resident A and G)."""
    _fullsize(128, "patch")
