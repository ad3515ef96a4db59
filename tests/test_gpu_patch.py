"""GPU parity of the patch extension (ext_mode "patch": every column of P is
the least-energy extension of its R^T column into a patch of interior DoFs)
against the oracle's patch form, through the C ABI.

Integers (patches, every level) bit-exact.  Each column solves its own SPD
patch system, by Cholesky on the GPU and by LU in the oracle, so a column
agrees to c kappa(A_SS) eps relative to its largest entry; Galerkin
operators, the V-cycle and PCG follow with the tolerances of the block form."""
import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle
from gen import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2602_23613_amd as amglib   # noqa: E402

EPS = np.finfo(np.float64).eps
OPTS = dict(ext_mode="patch", patch_hops=2, patch_cap=128)

CASES = {
    "hex8_iso": dict(kind="hex", size=8, beta=1.0, alpha=1.0, seed=1),
    "hex12_jump": dict(kind="hex", size=12, beta=1.0,
                       alpha=lambda m: fields.subdomain_log_uniform(m, 4, 2), seed=102),
    "hex16_jump_b1e-3": dict(kind="hex", size=16, beta=1e-3,
                             alpha=lambda m: fields.subdomain_log_uniform(m, 8, 3), seed=103),
    "tri5_stripes": dict(kind="tri", size=5, beta=0.01, alpha=lambda m: fields.stripes_2d(m), seed=5),
    "tet5_checker": dict(kind="tet", size=5, beta=1e-2, alpha=lambda m: fields.checkerboard(m, 2),
                         seed=104, jitter=0.2, mesh_seed=4),
}
_cache = {}


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def case(name):
    if name not in _cache:
        c = dict(CASES[name])
        kw = {k: c.pop(k) for k in ("jitter", "mesh_seed") if k in c}
        seed = c.pop("seed")
        p = gen.make_problem(c["kind"], c["size"], alpha=c["alpha"], beta=c["beta"],
                             f=lambda n: fields.rhs_uniform(n, seed), **kw)
        Ho = oracle.setup(p.A, p.G, **OPTS)
        _cache[name] = (p, Ho)
    return _cache[name]


def patch_kappa(Ho, l):
    lv = Ho.levels[l]
    A = lv.A.tocsr()
    return max([np.linalg.cond(A[S][:, S].toarray()) for S in lv.patches if len(S)] or [1.0])


def level_kappa(Ho, l):
    lv = Ho.levels[l]
    ks = max([np.linalg.cond(L @ L.T) for L in lv.smoother.chol] or [1.0])
    return max(patch_kappa(Ho, l), ks)


def hier_kappa(Ho):
    if not hasattr(Ho, "_kp"):
        Ho._kp = max(level_kappa(Ho, l) for l in range(Ho.nlevels - 1))
    return Ho._kp


@pytest.mark.parametrize("name", list(CASES))
def test_patch_hierarchy_integers_bit_exact(name):
    dev()
    p, Ho = case(name)
    H = amglib.Hierarchy(p.A, p.G, **OPTS)
    info = H.info()
    assert [l["n"] for l in info] == [l.A.shape[0] for l in Ho.levels]
    assert [l["nnz"] for l in info] == [l.A.nnz for l in Ho.levels]
    for l in range(len(Ho.levels) - 1):
        d = H.integers(l)
        lv = Ho.levels[l]
        ptr = np.concatenate([[0], np.cumsum([len(x) for x in lv.patches])])
        assert np.array_equal(d["patch_ptr"], ptr), l
        assert np.array_equal(d["patch_dofs"], np.concatenate(lv.patches)), l
        for f in ("dof1", "dof2", "s1", "s2"):
            assert np.array_equal(d["r_" + f], getattr(lv.rr, f)), f
    H.close()


@pytest.mark.parametrize("name", list(CASES))
def test_patch_interpolation_and_galerkin_values(name):
    dev()
    p, Ho = case(name)
    H = amglib.Hierarchy(p.A, p.G, **OPTS)
    for l in range(len(Ho.levels) - 1):
        A_l, P_l = H.level(l)
        A_n, _ = H.level(l + 1)
        lv = Ho.levels[l]
        assert np.array_equal(P_l.indptr, lv.P.indptr) and np.array_equal(P_l.indices, lv.P.indices)
        k = patch_kappa(Ho, l)
        # on coarse levels both sides solve with their own Galerkin A_l, which
        # differ by delta relative to A_l's row maxima: the patch solves then
        # agree to kappa (eps + delta)
        rmax = np.asarray(abs(lv.A).max(axis=1).todense()).ravel()
        rows_l = np.repeat(np.arange(lv.A.shape[0]), np.diff(lv.A.indptr))
        delta = float(np.max(np.abs(A_l.data - lv.A.data) / rmax[rows_l]))
        # column by column, relative to the column's largest entry
        Pg = sp.csc_matrix(P_l)
        Po = sp.csc_matrix(lv.P)
        D = abs(Pg - Po).max(axis=0).toarray().ravel()
        M = abs(Po).max(axis=0).toarray().ravel()
        eP = float(np.max(D / np.maximum(M, 1e-300)))
        absP = abs(lv.P)
        S = (absP.T @ abs(lv.A) @ absP).tocsr()
        Ao = Ho.levels[l + 1].A
        assert np.array_equal(A_n.indptr, Ao.indptr) and np.array_equal(A_n.indices, Ao.indices)
        scale = np.asarray(S.max(axis=1).todense()).ravel()
        rows = np.repeat(np.arange(Ao.shape[0]), np.diff(Ao.indptr))
        eA = float(np.max(np.abs(A_n.data - Ao.data) / scale[rows]))
        print(f"level {l}: patch kappa {k:.1e}  A_l delta {delta:.1e}  P err {eP:.1e}  "
              f"A_c err {eA:.1e}")
        assert eP <= max(1e-13, 8 * k * (EPS + delta)), (l, eP)
        assert eA <= max(1e-13, 16 * k * (EPS + delta)), (l, eA)
    H.close()


@pytest.mark.parametrize("name", list(CASES))
def test_patch_vcycle_matches_oracle(name):
    d = dev()
    p, Ho = case(name)
    H = amglib.Hierarchy(p.A, p.G, **OPTS)
    r = np.random.default_rng(21).standard_normal(p.A.shape[0])
    rt = torch.tensor(r, device=d)
    zt = torch.zeros_like(rt)
    H.vcycle(rt, zt)
    torch.cuda.synchronize()
    zo = oracle.vcycle(Ho, r)
    err = np.linalg.norm(zt.cpu().numpy() - zo) / np.linalg.norm(zo)
    tol = max(1e-10, 16 * hier_kappa(Ho) * EPS)
    print(f"patch V-cycle rel err {err:.2e} (tol {tol:.1e})")
    assert err <= tol
    H.close()


@pytest.mark.parametrize("name", list(CASES))
def test_patch_pcg_matches_oracle(name):
    d = dev()
    p, Ho = case(name)
    H = amglib.Hierarchy(p.A, p.G, **OPTS)
    f = torch.tensor(p.f, device=d)
    u = torch.zeros_like(f)
    st = H.pcg(f, u, rtol=1e-8, maxit=500, history=True)
    xo, it_o, hist_o = oracle.pcg(Ho, p.A, p.f, maxit=500)
    first_g = int(np.argmax(st["history"] <= 1e-8 * st["history"][0]))
    first_o = int(np.argmax(np.asarray(hist_o) <= 1e-8 * hist_o[0]))
    print(f"patch PCG its {st['iterations']} (oracle {it_o}), first crossing {first_g} / {first_o}")
    assert abs(first_g - first_o) <= 1, (first_g, first_o)
    assert st["converged"] == (st["true_relres"] <= 1e-8)
    uu = u.cpu().numpy()
    floor = 64 * EPS * np.linalg.norm(abs(p.A) @ np.abs(uu)) / np.linalg.norm(p.f)
    assert st["true_relres"] <= max(2e-8, floor)
    H.close()


def test_patch_numeric_resetup_matches_fresh_setup():
    """amg_resetup_numeric in the patch form (new coefficient field, same
    pattern: the patches and every integer result are reused) gives the
    same V-cycle bits as a fresh setup on the new field, and repeated
    V-cycles are bitwise equal."""
    d = dev()
    p1 = gen.make_problem("hex", 10, alpha=lambda m: fields.subdomain_log_uniform(m, 5, 21))
    p2 = gen.make_problem("hex", 10, alpha=lambda m: fields.subdomain_log_uniform(m, 5, 22))
    H = amglib.Hierarchy(p1.A, p1.G, **OPTS)
    H.resetup(p2.A)
    H2 = amglib.Hierarchy(p2.A, p2.G, **OPTS)
    r = torch.tensor(np.random.default_rng(3).standard_normal(p1.A.shape[0]), device=d)
    z1, z2, z3 = torch.zeros_like(r), torch.zeros_like(r), torch.zeros_like(r)
    H.vcycle(r, z1)
    H2.vcycle(r, z2)
    H2.vcycle(r, z3)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    assert torch.equal(z2, z3)
    H.close()
    H2.close()


def test_patch_mode_rejects_the_learned_setup():
    """The network predicts block solves: the patch form refuses to train it."""
    dev()
    p, _ = case("hex8_iso")
    H = amglib.Hierarchy(p.A, p.G, **OPTS)
    with pytest.raises(amglib.AmgError):
        H.mlp_train(epochs=1, batch=64)
    H.close()
