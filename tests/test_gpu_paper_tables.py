"""The paper's own 2D workloads on the GPU path (Section 5, Tables 1-2), the
stand-alone cycle iteration, the smoothing orders and the caller-given
("Geo") interpolation, against the CPU oracle.

Tables 1-2 use a random initial guess (seed 0) and b = (1, ..., n); beta =
0.01; tolerance 1e-8.  The GPU hierarchies' operator complexities must equal
the printed ones to every digit, and the iteration counts must equal the
oracle's (within one: both sides round differently).  Every call goes
through the C ABI."""
import json
import os

import numpy as np
import pytest

import gen
import oracle
from gen import fields
from refsel import RefSelector

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2602_23613_amd as amglib   # noqa: E402

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables_1_2.json")))
EPS = np.finfo(np.float64).eps


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _ref_lists(p, L):
    """Coarse node lists of the refinement hierarchy per level (the same
    selector the oracle uses, replayed on the oracle's levels)."""
    sel = RefSelector(p)
    Ho = oracle.setup(p.A, p.G, interp="ref", ref_select=sel, max_levels=L, min_coarse=0)
    sel2 = RefSelector(p)
    return [sel2(l, Ho.levels[l]) for l in range(Ho.nlevels - 1)]


def _pair(p, L, interp, schwarz):
    """(GPU hierarchy, oracle hierarchy) of one Table 1-2 column."""
    if interp == "ref":
        Ho = oracle.setup(p.A, p.G, interp="ref", ref_select=RefSelector(p), max_levels=L,
                          min_coarse=0, schwarz=schwarz)
        H = amglib.Hierarchy(p.A, p.G, interp="ref", ref=_ref_lists(p, L), max_levels=L,
                             min_coarse=0, schwarz=schwarz)
    elif interp == "geo":
        Ps, Gs = gen.geo_hierarchy("tri", L, L)
        Ho = oracle.setup(p.A, p.G, user=(Ps, Gs), schwarz=schwarz)
        H = amglib.Hierarchy(p.A, p.G, interp="user", user=(Ps, Gs), schwarz=schwarz)
    else:
        Ho = oracle.setup(p.A, p.G, schwarz=schwarz)
        H = amglib.Hierarchy(p.A, p.G, schwarz=schwarz)
    return H, Ho


@pytest.mark.parametrize("table,L", [("table1", 4), ("table1", 5), ("table2", 4), ("table2", 5)])
@pytest.mark.parametrize("interp", ["geo", "ref", "alg"])
def test_paper_table_counts_on_gpu(table, L, interp):
    d = dev()
    alpha = 1.0 if table == "table1" else (lambda m: fields.stripes_2d(m))
    p = gen.make_problem("tri", L, beta=0.01, alpha=alpha)
    n = p.A.shape[0]
    b = np.arange(1, n + 1, dtype=float)
    x0 = np.random.default_rng(0).random(n)
    key = "table1_uniform_isotropic" if table == "table1" else "table2_uniform_stripes"
    row = GOLDEN[key][str(L)]
    out = {}
    for schwarz in ("adjoint", "repeat"):
        H, Ho = _pair(p, L, interp, schwarz)
        oc, gc = H.complexity()
        assert abs(oc - row["oc_" + ("ref" if interp == "geo" else interp)]) < 1e-12
        assert abs(oc - Ho.oc()) < 1e-12 and abs(gc - Ho.gc()) < 1e-12
        bt = torch.tensor(b, device=d)
        if schwarz == "adjoint":
            u = torch.tensor(x0, device=d)
            st = H.pcg(bt, u, rtol=1e-8, maxit=500)
            _, it_o, _ = oracle.pcg(Ho, p.A, b, x0=x0)
            assert st["converged"] and abs(st["iterations"] - it_o) <= 1, (st, it_o)
            out["pcg"] = (st["iterations"], it_o)
        u = torch.tensor(x0, device=d)
        st = H.cycle_solve(bt, u, rtol=1e-8, maxit=400)
        _, ita_o, h = oracle.amg_solve(Ho, p.A, b, x0=x0)
        assert abs(st["iterations"] - ita_o) <= 1, (schwarz, st["iterations"], ita_o)
        assert abs(st["conv_factor"] - h[-1] / h[-2]) <= 0.01
        out["amg_" + schwarz] = (st["iterations"], ita_o, round(st["conv_factor"], 4))
        H.close()
    print(table, L, interp, out)


@pytest.mark.parametrize("schwarz", ["repeat", "split"])
@pytest.mark.parametrize("name", ["hex12_jump", "tri5_stripes"])
def test_smoothing_orders_match_oracle(schwarz, name):
    """The cycle with the other smoothing orders of Section 5's OSS-l1 step
    (post = pre; fwd-pre / bwd-post) against the oracle."""
    import test_gpu_parity as tp
    d = dev()
    p, _ = tp.case(name)
    Ho = oracle.setup(p.A, p.G, schwarz=schwarz)
    H = amglib.Hierarchy(p.A, p.G, schwarz=schwarz)
    r = np.random.default_rng(2).standard_normal(p.A.shape[0])
    rt = torch.tensor(r, device=d)
    zt = torch.zeros_like(rt)
    H.vcycle(rt, zt)
    torch.cuda.synchronize()
    zo = oracle.vcycle(Ho, r)
    err = np.linalg.norm(zt.cpu().numpy() - zo) / np.linalg.norm(zo)
    tol = max(1e-10, 16 * tp.kappas(tp.case(name)[1])[1] * EPS)
    print(f"{schwarz}: V-cycle rel err {err:.2e} (tol {tol:.1e})")
    assert err <= tol
    H.close()


def test_geo_interpolation_hex_jumps_on_gpu():
    """The geometric Nedelec hierarchy of a 16^3 hex jump problem through the
    caller-given interpolation mode: A_c, the V-cycle and PCG against the
    oracle (the comparison method of Section 5 in 3D)."""
    d = dev()
    N = 16
    p = gen.make_problem("hex", N, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 8, 2),
                         f=lambda n: fields.rhs_uniform(n, 102))
    Ps, Gs = gen.geo_hierarchy("hex", N, 4)
    Ho = oracle.setup(p.A, p.G, user=(Ps, Gs))
    H = amglib.Hierarchy(p.A, p.G, interp="user", user=(Ps, Gs))
    info = H.info()
    assert [l["n"] for l in info] == [lv.A.shape[0] for lv in Ho.levels]
    for l in range(1, len(info)):
        A_l, _ = H.level(l)
        Ao = Ho.levels[l].A
        assert np.array_equal(A_l.indptr, Ao.indptr) and np.array_equal(A_l.indices, Ao.indices)
        assert np.abs(A_l.data - Ao.data).max() <= 1e-12 * np.abs(Ao.data).max()
    r = np.random.default_rng(4).standard_normal(p.A.shape[0])
    rt = torch.tensor(r, device=d)
    zt = torch.zeros_like(rt)
    H.vcycle(rt, zt)
    torch.cuda.synchronize()
    zo = oracle.vcycle(Ho, r)
    import test_gpu_parity as tp
    tol = max(1e-10, 16 * max(tp.kappa_level(Ho, l) for l in range(Ho.nlevels - 1)) * EPS)
    err = np.linalg.norm(zt.cpu().numpy() - zo) / np.linalg.norm(zo)
    assert err <= tol, (err, tol)
    f = torch.tensor(p.f, device=d)
    u = torch.zeros_like(f)
    st = H.pcg(f, u, rtol=1e-8, maxit=2000)
    _, it_o, hist = oracle.pcg(Ho, p.A, p.f, maxit=2000)
    print(f"Geo 16^3 jumps: PCG {st['iterations']} (oracle {it_o}), V-cycle err {err:.1e}")
    assert st["true_relres"] <= max(2e-8, st["floor_relres"])
    assert abs(st["iterations"] - it_o) <= max(3, 0.1 * it_o)
    H.close()


def test_user_interpolation_rejects_bad_shapes():
    dev()
    p = gen.make_problem("tri", 3, beta=0.01)
    Ps, Gs = gen.geo_hierarchy("tri", 3, 3)
    with pytest.raises(amglib.AmgError):
        amglib.Hierarchy(p.A, p.G, interp="user", user=([Ps[1]], Gs))
    with pytest.raises(amglib.AmgError):
        amglib.Hierarchy(p.A, p.G, interp="user", user=(Ps, [Gs[0], Gs[2], Gs[1]]))
