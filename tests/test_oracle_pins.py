"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: they check closed forms,
theorems of the paper, printed table values, brute force and invariants.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import gen
import oracle
from oracle import amg
from gen import fields
from refsel import RefSelector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables_1_2.json")


# ----------------------------------------------------------------------------
# inputs: Nedelec assembly (Section 2)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("kind,size,kw", [("hex", 3, {}), ("hex", 5, {}), ("tri", 3, {}),
                                          ("tet", 3, dict(jitter=0.2, mesh_seed=4))])
def test_curl_part_annihilates_gradients(kind, size, kw):
    """ker A^s = range G (de Rham, Section 2)."""
    p = gen.make_problem(kind, size, alpha=lambda m: fields.subdomain_log_uniform(m, 2, 7),
                         parts=True, **kw)
    assert abs(p.As @ p.G).max() <= 1e-12 * abs(p.As).max()
    # and the mass part does not: A is SPD, G has full column rank
    assert abs(p.Am @ p.G).max() > 1e-3 * abs(p.Am).max()


def test_dof_counts_closed_forms():
    # hex, Dirichlet: 3N(N-1)^2 DoFs; natural: 3N(N+1)^2
    for N in (2, 4, 8):
        p = gen.make_problem("hex", N)
        assert p.A.shape[0] == 3 * N * (N - 1) ** 2
    assert gen.make_problem("hex", 8).A.nnz == 31008
    assert gen.make_problem("hex", 8, dirichlet=False).A.shape[0] == 1944
    # uniform triangles, Dirichlet: n = 3 4^L - 2 2^L, nnz = 15 4^L - 18 2^L + 4
    for L in (2, 3, 4, 5):
        p = gen.make_problem("tri", L)
        assert p.A.shape[0] == 3 * 4 ** L - 2 * 2 ** L
        assert p.A.nnz == 15 * 4 ** L - 18 * 2 ** L + 4
    # the sizes of Tables 1-2 (Section 5): 736, 3008, 12160 for L = 4, 5, 6
    assert [3 * 4 ** L - 2 * 2 ** L for L in (4, 5, 6, 7, 8)] == [736, 3008, 12160, 48896, 196096]
    # Kuhn tets: every edge of the N^3 cubes, face and body diagonals
    m = gen.kuhn_tet_mesh(3)
    assert m.edges.shape[0] == 3 * 3 * 16 + 3 * 9 * 4 + 27


def _edge_dofs_of_field(mesh, a, b):
    x0 = mesh.coords[mesh.edges[:, 0]]
    x1 = mesh.coords[mesh.edges[:, 1]]
    mid = 0.5 * (x0 + x1)
    if mesh.dim == 3:
        u = a[None, :] + np.cross(b[None, :], mid)
    else:
        u = a[None, :] + b * np.stack([-mid[:, 1], mid[:, 0]], axis=1)
    return np.einsum("ed,ed->e", u, x1 - x0)


@pytest.mark.parametrize("kind,size", [("hex", 3), ("tri", 3), ("tet", 2)])
def test_energies_of_rigid_fields(kind, size):
    """u = a + b x X lies in the lowest-order Nedelec space: curl u = 2b, so
    u^T A^s u = sum_K alpha_K |2b|^2 |K| and u^T A^m u = int |u|^2."""
    kw = dict(jitter=0.2, mesh_seed=3) if kind == "tet" else {}
    p = gen.make_problem(kind, size, alpha=lambda m: fields.subdomain_log_uniform(m, 2, 5, -1, 1),
                         dirichlet=False, parts=True, **kw)
    rng = np.random.default_rng(0)
    dim = p.mesh.dim
    a = rng.standard_normal(dim)
    b = rng.standard_normal(3) if dim == 3 else rng.standard_normal()
    u = _edge_dofs_of_field(p.mesh, a, b)
    vol = np.abs(amg_volumes(p.mesh))
    curl2 = 4.0 * (b @ b if dim == 3 else b * b)
    assert np.isclose(u @ (p.As @ u), np.sum(p.alpha * vol) * curl2, rtol=1e-12)
    # int |a + b x X|^2 over the unit square/cube, by a tensor Gauss rule (exact for quadratics)
    g = np.array([0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)])
    pts = np.array(np.meshgrid(*([g] * dim), indexing="ij")).reshape(dim, -1).T
    if dim == 3:
        uu = a[None] + np.cross(b[None], pts)
    else:
        uu = a[None] + b * np.stack([-pts[:, 1], pts[:, 0]], axis=1)
    exact = np.mean(np.sum(uu * uu, axis=1))
    assert np.isclose(u @ (p.Am @ u), exact, rtol=1e-12)


def amg_volumes(mesh):
    if mesh.kind == "hex":
        return np.full(mesh.elems.shape[0], mesh.h ** 3)
    X = mesh.coords[mesh.elems]
    J = np.stack([X[:, a + 1] - X[:, 0] for a in range(mesh.dim)], axis=2)
    return np.linalg.det(J) / (2.0 if mesh.dim == 2 else 6.0)


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------
def test_augment_g_hand_example():
    # 4 edges, 2 nodes: rows with one entry get a new column with the opposite sign
    G = sp.csr_matrix(np.array([[-1.0, 1.0], [0.0, 1.0], [-1.0, 0.0], [1.0, -1.0]]))
    Gt, B = amg.augment_g(G)
    want = np.array([[-1, 1, 0, 0], [0, 1, -1, 0], [-1, 0, 0, 1], [1, -1, 0, 0]], dtype=float)
    assert np.array_equal(Gt.toarray(), want)
    assert B.tolist() == [2, 3]


def test_augment_g_structure_hex():
    p = gen.make_problem("hex", 6)
    Gt, B = amg.augment_g(p.G)
    cnt = np.diff(Gt.indptr)
    assert np.all(cnt == 2)
    assert np.allclose(np.asarray(Gt.sum(axis=1)).ravel(), 0.0)
    # one artificial node per boundary-touching edge: 6 (N-1)^2
    assert len(B) == 6 * 25


# ----------------------------------------------------------------------------
# nodal graph, C/F splitting (Algorithm 2)
# ----------------------------------------------------------------------------
def test_nodal_graph_is_27_point_on_hex():
    N = 6
    p = gen.make_problem("hex", N)
    Gt, B = amg.augment_g(p.G)
    S = amg.nodal_graph(p.A, Gt)
    m = p.G.shape[1]
    deg = np.diff(S.indptr)[:m]
    # interior nodes not next to the boundary have the 26 king-move neighbours
    ijk = np.array(np.unravel_index(np.arange(m), (N - 1,) * 3))  # k, j, i of interior lattice
    deep = np.all((ijk >= 1) & (ijk <= N - 3), axis=0)
    assert np.all(deg[deep] == 26)


def test_rs_splitting_invariants_and_hex_lattice():
    for N in (6, 8, 10):
        p = gen.make_problem("hex", N)
        Gt, B = amg.augment_g(p.G)
        S = amg.nodal_graph(p.A, Gt)
        cG, st = amg.nodal_cf(S, B)
        isC = st == 1
        isB = np.zeros(S.shape[0], dtype=bool)
        isB[B] = True
        # no chosen C node next to another C node (the prescribed boundary nodes
        # B may touch each other); every node decided; every F has a C neighbour
        rows = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr))
        assert not np.any(isC[rows] & ~isB[rows] & isC[S.indices])
        assert np.all(st != 0)
        hasC = np.zeros(S.shape[0], dtype=bool)
        np.logical_or.at(hasC, rows, isC[S.indices])
        assert np.all(hasC[st == 2])
        # closed form: coarse nodes are the even interior lattice ((N/2-1)^3 nodes)
        m = p.G.shape[1]
        lat = np.array(np.unravel_index(np.arange(m), (N - 1,) * 3)) + 1
        even = np.nonzero(np.all(lat % 2 == 0, axis=0))[0]
        assert np.array_equal(cG, even)


# ----------------------------------------------------------------------------
# Algorithm 3
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("kind,size", [("tri", 3), ("hex", 4), ("hex", 6), ("tet", 3)])
def test_matching_postconditions_brute_force(kind, size):
    """Every DoF in at most one R row; every middle node used once; r G~ = -e_i + e_j;
    R R^T = 2 I; R S_I = 0; and (brute force over all pairs of C') every pair at
    edge distance exactly two, not both in B, is either matched or blocked
    because its smallest mutual neighbour is already a middle."""
    kw = dict(jitter=0.2, mesh_seed=4) if kind == "tet" else {}
    p = gen.make_problem(kind, size, **kw)
    Gt, B = amg.augment_g(p.G)
    S = amg.nodal_graph(p.A, Gt)
    cG, _ = amg.nodal_cf(S, B)
    Cp = np.concatenate([cG, B])
    n = p.A.shape[0]
    rr, interior = amg.form_r(Gt, Cp, B, n)
    dofs = np.concatenate([rr.dof1, rr.dof2])
    assert len(np.unique(dofs)) == len(dofs)
    assert len(np.unique(rr.k)) == len(rr.k)
    R = amg.r_transpose(rr, n).T.tocsr()
    RG = (R @ Gt).toarray()
    want = np.zeros_like(RG)
    want[np.arange(len(rr)), rr.i] = -1
    want[np.arange(len(rr)), rr.j] = 1
    assert np.array_equal(RG, want)
    assert np.array_equal((R @ R.T).toarray(), 2 * np.eye(len(rr)))
    assert abs(R[:, interior]).sum() == 0
    assert np.array_equal(np.sort(np.concatenate([dofs, interior])), np.arange(n))
    # brute force over all pairs
    E, _ = amg.edge_graph(Gt)
    D = shortest_path(E, unweighted=True, indices=Cp)
    Cset = np.sort(Cp)
    isB = np.zeros(Gt.shape[1], dtype=bool)
    isB[B] = True
    matched = set(zip(np.minimum(rr.i, rr.j).tolist(), np.maximum(rr.i, rr.j).tolist()))
    K = set(rr.k.tolist())
    Ed = E.toarray() > 0
    pos = {c: t for t, c in enumerate(Cp)}
    for a in Cset:
        for b in Cset:
            if b <= a or (isB[a] and isB[b]) or D[pos[a], b] != 2:
                continue
            kmin = int(np.nonzero(Ed[a] & Ed[b])[0][0])
            assert (a, b) in matched or kmin in K
    # hex: the pairs are exactly the coarse-mesh edges of the refinement
    if kind == "hex":
        N = size
        assert len(rr) == 3 * (N // 2) * (N // 2 - 1) ** 2


# ----------------------------------------------------------------------------
# Tables 1-2: structural complexities (Section 5)
# ----------------------------------------------------------------------------
def _golden():
    return json.load(open(GOLDEN))


@pytest.mark.parametrize("L", [4, 5, 6])
def test_table1_algebraic_complexities_exact(L):
    """Alg: the operator and grid complexities and level counts printed in
    Table 1 (and, identically, Table 2) are reproduced to every digit."""
    row = _golden()["table1_uniform_isotropic"][str(L)]
    for alpha in (1.0, lambda m: fields.stripes_2d(m)):
        p = gen.make_problem("tri", L, beta=0.01, alpha=alpha)
        H = oracle.setup(p.A, p.G)
        assert H.nlevels == row["levels_alg"]
        assert abs(H.oc() - row["oc_alg"]) < 1e-12
        assert abs(H.gc() - row["gc_alg"]) < 1e-12


@pytest.mark.parametrize("L", [4, 5, 6])
def test_table1_refinement_complexities_exact(L):
    """Ref (coarse nodes from the geometric hierarchy): Table 1's OC/GC."""
    row = _golden()["table1_uniform_isotropic"][str(L)]
    p = gen.make_problem("tri", L, beta=0.01)
    H = oracle.setup(p.A, p.G, interp="ref", ref_select=RefSelector(p), max_levels=L, min_coarse=0)
    assert H.nlevels == row["levels_ref"]
    assert abs(H.oc() - row["oc_ref"]) < 1e-12
    assert abs(H.gc() - row["gc_ref"]) < 1e-12


def _table_hier(p, L, interp, schwarz):
    if interp == "ref":
        return oracle.setup(p.A, p.G, interp="ref", ref_select=RefSelector(p), max_levels=L,
                            min_coarse=0, schwarz=schwarz)
    if interp == "geo":
        return oracle.setup(p.A, p.G, user=gen.geo_hierarchy("tri", L, L), schwarz=schwarz)
    return oracle.setup(p.A, p.G, schwarz=schwarz)


def _table_run(L, alpha, interp, schwarz):
    """Section 5's protocol: random x0 (seed 0), b = (1..n), tolerance 1e-8."""
    p = gen.make_problem("tri", L, beta=0.01, alpha=alpha)
    n = p.A.shape[0]
    b = np.arange(1, n + 1, dtype=float)
    x0 = np.random.default_rng(0).random(n)
    H = _table_hier(p, L, interp, schwarz)
    _, it, _ = oracle.pcg(H, p.A, b, x0=x0)
    _, ita, h = oracle.amg_solve(H, p.A, b, x0=x0)
    return H, it, ita, h[-1] / h[-2]


@pytest.mark.parametrize("L", [4, 5, 6])
def test_table1_iteration_counts_all_three_interpolations(L):
    """Table 1 (isotropic), Geo / Ref / Alg:
    * OC to every printed digit (Geo's from the Galerkin products of the
      geometric interpolation, which pins that P's pattern and levels);
    * PCG counts within one, with the symmetric (adjoint) cycle;
    * stand-alone AMG ("AMG conv": ratio of the last two residuals) within
      0.02 of the printed factor, with the literal cycle (post step = pre
      step); AMG counts within one for Geo and Ref, within three for Alg."""
    row = _golden()["table1_uniform_isotropic"][str(L)]
    conv = _golden()["table1_amg_conv"][str(L)]
    for interp in ("geo", "ref", "alg"):
        key = "ref" if interp == "geo" else interp      # Table 1 prints Geo = Ref
        H, it, _, _ = _table_run(L, 1.0, interp, "adjoint")
        assert abs(H.oc() - row["oc_" + key]) < 1e-12, interp
        assert abs(it - row["pcg_" + key]) <= 1, (interp, it)
        _, _, ita, rho = _table_run(L, 1.0, interp, "repeat")
        assert abs(rho - conv[key]) <= 0.02, (interp, rho)
        assert abs(ita - row["amg_" + key]) <= (3 if interp == "alg" else 1), (interp, ita)


@pytest.mark.parametrize("L", [4, 5])
def test_table2_algebraic_counts(L):
    """Table 2 (stripes), Alg: OC to every digit, the AMG convergence factor
    within 0.01 of the printed one (literal cycle), PCG within two."""
    row = _golden()["table2_uniform_stripes"][str(L)]
    conv = _golden()["table2_amg_conv"][str(L)]
    stripes = lambda m: fields.stripes_2d(m)
    H, it, _, _ = _table_run(L, stripes, "alg", "adjoint")
    assert abs(H.oc() - row["oc_alg"]) < 1e-12
    assert abs(it - row["pcg_alg"]) <= 2
    _, _, ita, rho = _table_run(L, stripes, "alg", "repeat")
    assert abs(rho - conv["alg"]) <= 0.01, rho


@pytest.mark.parametrize("L", [4, 5])
def test_table2_ref_and_geo_are_not_reproduced(L):
    """Table 2 Ref (AMG 8-13, PCG 5) and Geo (AMG 80-320) are NOT reproduced
    by the node-star smoother reading: the oracle converges at ~0.55-0.62 on
    Ref (printed 0.17-0.32) and ~0.95 on Geo (printed 0.84-0.96).  No other
    reading tried reproduces them either (element-patch blocks, blocks from
    the matching, other stripe layouts); with the same geometric P, printed
    Table 1 and the Table 2 Alg column are reproduced.  This test records the
    oracle's values so that a change of reading shows up here."""
    rec = _golden()["oracle_table2_record"][str(L)]
    stripes = lambda m: fields.stripes_2d(m)
    for interp in ("ref", "geo"):
        H, it, _, _ = _table_run(L, stripes, interp, "adjoint")
        _, _, ita, rho = _table_run(L, stripes, interp, "repeat")
        assert abs(H.oc() - _golden()["table2_uniform_stripes"][str(L)]["oc_ref"]) < 1e-12
        assert it == rec[interp]["pcg"] and ita == rec[interp]["amg"], (interp, it, ita)
        assert abs(rho - rec[interp]["amg_conv"]) < 1e-3


@pytest.mark.parametrize("L", [4, 5])
def test_smoother_readings_against_tables_1_and_2(L):
    """Neither smoother reading reproduces both tables.  Node stars (the
    reading the library uses) reproduce Table 1 (all three columns) and the
    Table 2 Alg column, but not Table 2 Ref.  Node stars plus the interior
    blocks of each level's splitting (the decoupled fine-variable blocks of
    the matching) reproduce Table 2 Ref at L = 4 (AMG 8, PCG 6 against the
    printed 8 and 5) but stay at AMG 8 where the paper prints 11, and they
    break Table 1 (AMG 9 against the printed 22).  Both readings' counts are
    recorded so that a change of either shows up here."""
    g = _golden()
    rec = g["oracle_record_stars_interior"][str(L)]
    stripes = lambda m: fields.stripes_2d(m)
    for interp in ("ref", "alg"):
        for tab, al in (("table2", stripes), ("table1", 1.0)):
            p = gen.make_problem("tri", L, beta=0.01, alpha=al)
            n = p.A.shape[0]
            b = np.arange(1, n + 1, dtype=float)
            x0 = np.random.default_rng(0).random(n)
            kw = dict(interp="ref", ref_select=RefSelector(p), max_levels=L, min_coarse=0) \
                if interp == "ref" else {}
            H = oracle.setup(p.A, p.G, smoother_blocks="stars+interior", schwarz="adjoint", **kw)
            _, it, _ = oracle.pcg(H, p.A, b, x0=x0)
            kw2 = dict(kw, ref_select=RefSelector(p)) if interp == "ref" else {}
            H = oracle.setup(p.A, p.G, smoother_blocks="stars+interior", schwarz="repeat", **kw2)
            _, ita, h = oracle.amg_solve(H, p.A, b, x0=x0)
            r = rec[f"{tab}_{interp}"]
            assert (it, ita) == (r["pcg"], r["amg"]), (tab, interp, it, ita)
            assert abs(h[-1] / h[-2] - r["amg_conv"]) < 1e-3
    printed2 = g["table2_uniform_stripes"][str(L)]
    printed1 = g["table1_uniform_isotropic"][str(L)]
    # what each reading matches
    assert abs(rec["table2_ref"]["amg"] - printed2["amg_ref"]) <= (2 if L == 4 else 3)
    assert abs(rec["table1_ref"]["amg"] - printed1["amg_ref"]) > 10
    stars = g["oracle_table2_record"][str(L)]["ref"]
    assert abs(stars["amg"] - printed2["amg_ref"]) > 10


# ----------------------------------------------------------------------------
# interpolation, theory (Section 3)
# ----------------------------------------------------------------------------
def _two_level_2d(L=3, beta=0.01, alpha=1.0, As_only=False):
    """Refinement-based R and P_app of the finest level (no smoother, so that
    A = A^s, whose node-star blocks are singular, can be used)."""
    p = gen.make_problem("tri", L, beta=beta, alpha=alpha, parts=True)
    A = p.As if As_only else p.A
    lv = amg.Level(A=sp.csr_matrix(A), G=p.G)
    lv.Gt, lv.B = amg.augment_g(p.G)
    cG, Bc = RefSelector(p)(0, lv)
    Cp = np.concatenate([cG, Bc])
    n = A.shape[0]
    lv.rr, lv.interior = amg.form_r(lv.Gt, Cp, lv.B, n, skip_bb=False)
    lv.blocks, lv.depths, lv.exact_blocks = amg.extension_blocks(
        lv.A, lv.Gt, lv.interior, np.concatenate([Cp, lv.rr.k]))
    lv.P = amg.interpolation(lv.A, amg.r_transpose(lv.rr, n), lv.blocks, lv.depths)
    return p, A, lv


def test_block_extension_equals_dense_ideal_formula():
    """2D: graph(A_II) splits into small components, and P equals
    R^T - S_I A_II^{-1} S_I^T A R^T computed densely (eq. sparseP)."""
    for alpha in (1.0, lambda m: fields.stripes_2d(m)):
        for mode in ("ref", "alg"):
            p = gen.make_problem("tri", 3, beta=0.01, alpha=alpha)
            kw = dict(interp="ref", ref_select=RefSelector(p), min_coarse=0) if mode == "ref" else {}
            H = oracle.setup(p.A, p.G, max_levels=2, **kw)
            lv = H.levels[0]
            assert lv.exact_blocks
            n = p.A.shape[0]
            Rt = amg.r_transpose(lv.rr, n).toarray()
            Ad = p.A.toarray()
            I = lv.interior
            Pd = Rt.copy()
            Pd[I] = Rt[I] - np.linalg.solve(Ad[np.ix_(I, I)], Ad[I] @ Rt)
            assert np.abs(lv.P.toarray() - Pd).max() <= 1e-10 * np.abs(Pd).max()


def test_lemma1_and_commuting_theorem_2d():
    """beta = 0 (A = A^s, A^s_II invertible on the 2D refinement): Lemma 1
    X_E(A^s) S_E = 0 and X_E(A^s) G_E = 0, and Theorem 2: A^s P G_c = 0."""
    p, As, lv = _two_level_2d(L=3, alpha=lambda m: fields.stripes_2d(m), As_only=True)
    n = As.shape[0]
    Ad = As.toarray()
    I = lv.interior
    E = np.setdiff1d(np.arange(n), I)
    XE = Ad[np.ix_(E, E)] - Ad[np.ix_(E, I)] @ np.linalg.solve(Ad[np.ix_(I, I)], Ad[np.ix_(I, E)])
    # S_E: one column per R row, the oriented difference of its two DoFs
    SE = np.zeros((n, len(lv.rr)))
    SE[lv.rr.dof1, np.arange(len(lv.rr))] = lv.rr.s1
    SE[lv.rr.dof2, np.arange(len(lv.rr))] = -lv.rr.s2
    # S_E columns are the restrictions of G's columns at the middle nodes k
    scale = np.abs(XE).max()
    assert np.abs(XE @ SE[E]).max() <= 1e-10 * scale
    assert np.abs(XE @ p.G.toarray()[E]).max() <= 1e-10 * scale
    Gc, _ = amg.coarse_gradient(p.G, lv.rr)
    APG = As @ (lv.P @ Gc)
    assert abs(APG).max() <= 1e-10 * abs(As).max()


def test_commuting_defect_is_order_beta():
    """For beta != 0 the commuting relation holds up to O(beta): slope ~1 in log-log."""
    defects = []
    betas = [1e-1, 1e-2, 1e-3, 1e-4]
    for beta in betas:
        p, A, lv = _two_level_2d(L=3, beta=beta)
        Gc, _ = amg.coarse_gradient(p.G, lv.rr)
        defects.append(abs(p.As @ (lv.P @ Gc)).max())
    slopes = np.diff(np.log10(defects)) / np.diff(np.log10(betas))
    assert np.all(np.abs(slopes - 1.0) < 0.1)


def _coarse_hat_2d(xs, ys):
    """P1 hat of the unit '/'-cut square mesh centred at the origin."""
    return np.maximum.reduce([
        np.where((xs >= 0) & (ys >= 0) & (xs <= 1) & (ys <= 1), 1 - np.maximum(xs, ys), 0.0),
        np.where((xs <= 0) & (ys <= 0) & (xs >= -1) & (ys >= -1), 1 + np.minimum(xs, ys), 0.0),
        np.where((xs >= 0) & (ys <= 0) & (xs - ys <= 1), 1 - (xs - ys), 0.0),
        np.where((xs <= 0) & (ys >= 0) & (ys - xs <= 1), 1 - (ys - xs), 0.0)])


@pytest.mark.parametrize("alpha", [1.0, "stripes"])
def test_coarse_gradients_map_to_fine_gradients_of_linear_interpolant(alpha):
    """2D refinement (Section 3.1): P G_c / 2 = G P_n with P_n the piecewise
    linear interpolation of coarse nodal functions, up to O(beta) (the 1/2
    comes from the +-1 entries of R).  Checked for beta = 1e-2 and 1e-4."""
    al = (lambda m: fields.stripes_2d(m)) if alpha == "stripes" else alpha
    errs = []
    for beta in (1e-2, 1e-4):
        p, A, lv = _two_level_2d(L=3, beta=beta, alpha=al)
        Gc, cols = amg.coarse_gradient(p.G, lv.rr)
        M = 2 ** 3
        m = p.G.shape[1]
        lat = np.array(np.unravel_index(np.arange(m), (M - 1, M - 1)))[::-1] + 1   # (i, j)
        Pn = np.zeros((m, len(cols)))
        for c in range(len(cols)):
            Pn[:, c] = _coarse_hat_2d((lat[0] - lat[0, cols[c]]) / 2.0, (lat[1] - lat[1, cols[c]]) / 2.0)
        lhs = (lv.P @ Gc).toarray() / 2.0
        errs.append(np.abs(lhs - p.G.toarray() @ Pn).max())
    assert errs[1] < 1e-3 and errs[1] < errs[0] / 50


# ----------------------------------------------------------------------------
# Galerkin operator, smoother, cycle
# ----------------------------------------------------------------------------
def _small_hier():
    p = gen.make_problem("hex", 6, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 3, 11))
    return p, oracle.setup(p.A, p.G)


def test_galerkin_symmetric_positive_definite():
    p, H = _small_hier()
    for lv in H.levels[1:]:
        A = lv.A.toarray()
        assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


@pytest.mark.parametrize("kind,size,alpha", [("hex", 6, "jump"), ("tri", 4, "stripes")])
def test_l1_jacobi_diagonal_bounds_a(kind, size, alpha):
    """Section 5's l1-Jacobi divides by D_ii = sum_j |a_ij|.  D - A is then
    diagonally dominant with a non-negative diagonal, hence positive
    semi-definite (Gershgorin), so every eigenvalue of D^{-1} A lies in
    (0, 1] and the l1 step never increases the A-norm of the error.  The
    plain Jacobi diagonal diag(A) would put the largest one near 3 on
    these Nedelec matrices, so the pin tells the two apart."""
    import scipy.linalg as sl
    al = (lambda m: fields.subdomain_log_uniform(m, 2, 5)) if alpha == "jump" else \
        (lambda m: fields.stripes_2d(m))
    p = gen.make_problem(kind, size, beta=1.0, alpha=al)
    H = oracle.setup(p.A, p.G)
    assert H.nlevels >= 2
    for lv in H.levels[:-1]:
        A = lv.A.toarray()
        ev = sl.eigh(A, np.diag(lv.smoother.l1), eigvals_only=True)
        assert ev.min() > 0 and ev.max() <= 1 + 1e-12
        assert sl.eigh(A, np.diag(np.diag(A)), eigvals_only=True).max() > 2


@pytest.mark.parametrize("kind,size", [("hex", 6), ("tri", 4)])
def test_schwarz_colour_step_zeroes_the_residual_on_its_blocks(kind, size):
    """Section 5's multiplicative Schwarz solves each node-star block exactly:
    the blocks are the supports of the columns of G_l, and after one colour's
    step from any x the residual b - A x vanishes on every block of that
    colour (the blocks of a colour share no DoF and no entry of A, so one
    block's correction leaves the others' residuals alone)."""
    p = gen.make_problem(kind, size, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 2, 6)
                         if kind == "hex" else 1.0)
    H = oracle.setup(p.A, p.G)
    mats = amg._cast(H, np.float64)
    rng = np.random.default_rng(11)
    for l, lv in enumerate(H.levels[:-1]):
        G = sp.csc_matrix(lv.G)
        supports = [G.indices[G.indptr[v]:G.indptr[v + 1]] for v in range(G.shape[1])]
        stars = sorted(tuple(sorted(int(i) for i in sup)) for sup in supports if len(sup))
        assert sorted(tuple(int(i) for i in b) for b in lv.smoother.blocks) == stars
        A = sp.csr_matrix(lv.A)
        n = A.shape[0]
        for c in range(min(lv.smoother.ncolors, 4)):
            x = rng.standard_normal(n)
            b = rng.standard_normal(n)
            y = amg._schwarz(mats[l], x.copy(), b, [c])
            r = b - A @ y
            dofs = np.concatenate([blk for blk, col in zip(lv.smoother.blocks, lv.smoother.color)
                                   if col == c])
            scale = (abs(A) @ abs(y) + abs(b))[dofs].max()
            assert np.abs(r[dofs]).max() <= 1e-12 * scale
            others = np.setdiff1d(np.arange(n), dofs)
            assert np.array_equal(y[others], x[others])


def test_colouring_makes_colour_blocks_uncoupled():
    p, H = _small_hier()
    for lv in H.levels:
        sm = lv.smoother
        A = lv.A.tocsr()
        for c in range(sm.ncolors):
            owner = np.full(A.shape[0], -1)
            for b in np.nonzero(sm.color == c)[0]:
                assert np.all(owner[sm.blocks[b]] == -1)
                owner[sm.blocks[b]] = b
            for b in np.nonzero(sm.color == c)[0]:
                for e in sm.blocks[b]:
                    nb = owner[A.indices[A.indptr[e]:A.indptr[e + 1]]]
                    assert np.all((nb == -1) | (nb == b))


def test_colour_sweep_equals_sequential_block_sweep():
    """The colour-vectorised sweep equals block-by-block multiplicative Schwarz
    in colour order (written out directly with dense solves)."""
    p, H = _small_hier()
    lv = H.levels[0]
    sm = lv.smoother
    A = lv.A.tocsr()
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.shape[0])
    x = np.zeros_like(b)
    order = [blk for c in range(sm.ncolors) for blk in np.nonzero(sm.color == c)[0]]
    for blk in order:
        d = sm.blocks[blk]
        r = b[d] - A[d] @ x
        x[d] += np.linalg.solve(A[d][:, d].toarray(), r)
    mats = amg._cast(H, np.float64)
    y = amg._schwarz(mats[0], np.zeros_like(b), b, list(range(sm.ncolors)))
    assert np.abs(x - y).max() <= 1e-9 * np.abs(x).max()   # jumps of 10^8: local kappa ~1e7


def test_vcycle_is_symmetric_and_positive():
    p, H = _small_hier()
    rng = np.random.default_rng(1)
    n = p.A.shape[0]
    r1, r2 = rng.standard_normal(n), rng.standard_normal(n)
    v1, v2 = oracle.vcycle(H, r1), oracle.vcycle(H, r2)
    assert abs(v1 @ r2 - r1 @ v2) <= 1e-10 * np.linalg.norm(v1) * np.linalg.norm(r2)
    assert v1 @ r1 > 0


def test_two_grid_gamg_bound():
    """Section 1: ||E_TG||_A^2 <= 1 - 1/K with K = sup ||(I - P R^)e||^2_Mt / ||e||^2_A,
    Mt = M (M + M^T - A)^{-1} M^T, for any R^ with R^ P = I (here R^ = R/2).
    Checked densely on a tiny mesh with the oracle's own smoother."""
    for alpha in (1.0, lambda m: fields.subdomain_log_uniform(m, 2, 5)):
        p = gen.make_problem("hex", 4, beta=1.0, alpha=alpha)
        H = oracle.setup(p.A, p.G, max_levels=2)
        A = p.A.toarray()
        n = A.shape[0]
        lv = H.levels[0]
        P = lv.P.toarray()
        Rh = amg.r_transpose(lv.rr, n).toarray().T / 2.0
        assert np.allclose(Rh @ P, np.eye(P.shape[1]))
        # pre-smoother error propagation E_pre (columns = images of unit vectors)
        mats = amg._cast(H, np.float64)
        nc = lv.smoother.ncolors

        def pre(e):
            # smoothing A x = 0 from the initial error e gives the new error
            x = e.copy()
            b = np.zeros(n)
            x = amg._schwarz(mats[0], x, b, list(range(nc)))
            x = amg._schwarz(mats[0], x, b, list(range(nc - 1, -1, -1)))
            return x + (b - mats[0]["A"] @ x) / mats[0]["l1"]
        Epre = np.stack([pre(col) for col in np.eye(n)], axis=1)
        # M from I - M^{-1} A = E_pre
        M = A @ np.linalg.inv(np.eye(n) - Epre)
        Mt = M @ np.linalg.solve(M + M.T - A, M.T)
        Q = np.eye(n) - P @ Rh
        import scipy.linalg as sl
        K = sl.eigh(Q.T @ (0.5 * (Mt + Mt.T)) @ Q, A, eigvals_only=True).max()
        Pi = P @ np.linalg.solve(P.T @ A @ P, P.T @ A)
        E = Epre @ (np.eye(n) - Pi)
        # ||E||_A = ||A^{1/2} E A^{-1/2}||_2
        w, V = np.linalg.eigh(A)
        Ah = V @ np.diag(np.sqrt(w)) @ V.T
        Aih = V @ np.diag(1 / np.sqrt(w)) @ V.T
        nE = np.linalg.norm(Ah @ E @ Aih, 2)
        assert K >= 1.0
        assert nE ** 2 <= 1.0 - 1.0 / K + 1e-10


def test_pcg_reaches_tolerance_true_residual():
    p, H = _small_hier()
    f = fields.rhs_uniform(p.A.shape[0], 1)
    x, it, hist = oracle.pcg(H, p.A, f)
    assert np.linalg.norm(f - p.A @ x) <= 1.01e-8 * np.linalg.norm(f)
    assert it < 100


# ----------------------------------------------------------------------------
# geometric interpolation "Geo" (Section 5's comparison method; gen/geo.py)
# ----------------------------------------------------------------------------
def _rigid_dofs(mesh, a, b):
    x0 = mesh.coords[mesh.edges[:, 0]]
    x1 = mesh.coords[mesh.edges[:, 1]]
    mid = 0.5 * (x0 + x1)
    if mesh.dim == 3:
        u = a[None, :] + np.cross(b[None, :], mid)
    else:
        u = a[None, :] + b * np.stack([-mid[:, 1], mid[:, 0]], axis=1)
    return np.einsum("ed,ed->e", u, x1 - x0)


@pytest.mark.parametrize("kind,size", [("tri", 3), ("hex", 4)])
def test_geo_interpolation_reproduces_nedelec_fields(kind, size):
    """Nested spaces: a field a + b x X lies in the coarse and the fine
    Nedelec space, so interpolating its coarse DoFs gives its fine DoFs
    exactly (all edges kept)."""
    from gen import geo
    from gen.mesh import hex_mesh, simplex_mesh_2d
    fine = simplex_mesh_2d(size) if kind == "tri" else hex_mesh(size)
    coarse = simplex_mesh_2d(size - 1) if kind == "tri" else hex_mesh(size // 2)
    P = (geo.geo_interpolation_tri(size, dirichlet=False) if kind == "tri"
         else geo.geo_interpolation_hex(size, dirichlet=False))
    rng = np.random.default_rng(7)
    for _ in range(3):
        a = rng.standard_normal(fine.dim)
        b = rng.standard_normal(3) if fine.dim == 3 else rng.standard_normal()
        uc, uf = _rigid_dofs(coarse, a, b), _rigid_dofs(fine, a, b)
        assert np.abs(P @ uc - uf).max() <= 1e-13 * np.abs(uf).max()


def _nodal_interpolant(kind, fine, coarse, phi_c):
    """Fine nodal values of the P1 (triangles) / Q1 (hexahedra) interpolant of
    coarse nodal values: a fine node is a coarse node, or the midpoint of a
    coarse edge, face or cell, and takes the mean of that entity's vertices."""
    def key(x):
        return tuple(np.round(x * 2 ** 12).astype(np.int64))
    fidx = {key(c): i for i, c in enumerate(fine.coords)}
    out = np.full(fine.coords.shape[0], np.nan)
    if kind == "tri":
        groups = [coarse.edges]
    else:
        cells = coarse.elems                                   # 8 corners, bit a of the corner = offset in axis a
        faces = [cells[:, [c for c in range(8) if ((c >> ax) & 1) == side]]
                 for ax in range(3) for side in (0, 1)]
        groups = [coarse.edges, np.concatenate(faces), cells]
    for g in groups:
        for verts in g:
            out[fidx[key(coarse.coords[verts].mean(axis=0))]] = phi_c[verts].mean()
    for i, c in enumerate(coarse.coords):
        out[fidx[key(c)]] = phi_c[i]
    assert not np.isnan(out).any()
    return out


@pytest.mark.parametrize("kind,size", [("tri", 3), ("hex", 4)])
def test_geo_interpolation_commutes_with_nodal_interpolation(kind, size):
    """P_geo G_c = G P_n (eq. (commuting)) with P_n the nodal P1/Q1
    interpolation, on the Dirichlet spaces."""
    from gen import geo
    from gen.mesh import hex_mesh, simplex_mesh_2d
    fine = simplex_mesh_2d(size) if kind == "tri" else hex_mesh(size)
    coarse = simplex_mesh_2d(size - 1) if kind == "tri" else hex_mesh(size // 2)
    pf = gen.make_problem(kind, size)
    pc = gen.make_problem(kind, size - 1 if kind == "tri" else size // 2)
    P = geo.geo_interpolation_tri(size) if kind == "tri" else geo.geo_interpolation_hex(size)
    rng = np.random.default_rng(3)
    phi = np.zeros(coarse.coords.shape[0])
    phi[pc.keep_nodes] = rng.standard_normal(int(pc.keep_nodes.sum()))
    psi = _nodal_interpolant(kind, fine, coarse, phi)
    lhs = P @ (pc.G @ phi[pc.keep_nodes])
    rhs = pf.G @ psi[pf.keep_nodes]
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


# ----------------------------------------------------------------------------
# FP32 form: the per-level precision rule (parity unpinned by the paper)
# ----------------------------------------------------------------------------
def test_gradient_ratio_scales_like_alpha_over_beta():
    """rho = max_v (|G|^T |A| |G|)_vv / (G^T A G)_vv is scale-free and, as
    beta -> 0 (A^s G = 0, so only beta A^m sees a gradient), grows like 1/beta;
    the denominator is the energy of a hat gradient, hence positive."""
    r = {}
    for alpha, beta in ((1.0, 1.0), (10.0, 10.0), (1.0, 1e-2), (1.0, 1e-4)):
        p = gen.make_problem("hex", 4, alpha=alpha, beta=beta)
        assert np.all((p.G.T @ p.A @ p.G).diagonal() > 0)
        r[(alpha, beta)] = amg.gradient_ratio(p.A, p.G)
    assert abs(r[(10.0, 10.0)] / r[(1.0, 1.0)] - 1.0) < 1e-12
    assert abs(r[(1.0, 1e-4)] / r[(1.0, 1e-2)] - 100.0) < 1.0


def test_fp32_form_keeps_fp64_where_the_near_kernel_needs_it():
    """On the 16^3 jump workload (alpha up to 10^4, h = 1/16) eps_32 * rho is
    ~4 on the finest level, which therefore keeps FP64; the coarse levels
    run in FP32, and flexible CG reaches 1e-8 with such a cycle, while a cycle
    entirely in FP32 stalls (the FP32 residual loses the gradients)."""
    p = gen.make_problem("hex", 16, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 8, 2),
                         f=lambda n: fields.rhs_uniform(n, 102))
    H = oracle.setup(p.A, p.G)
    dts = amg.level_dtypes(H, np.float32)
    assert dts[0] == np.float64 and all(d == np.float32 for d in dts[1:-1])
    x, it, hist = oracle.pcg(H, p.A, p.f, dtype=np.float32, maxit=400)
    assert np.linalg.norm(p.f - p.A @ x) <= 1.01e-8 * np.linalg.norm(p.f) and it < 400
    H.opts["_level_dtypes"] = [np.float32] * H.nlevels
    x, it, hist = oracle.pcg(H, p.A, p.f, dtype=np.float32, maxit=150)
    assert np.linalg.norm(p.f - p.A @ x) > 1e-6 * np.linalg.norm(p.f)


@pytest.mark.parametrize("N,lo,hi", [(8, 2, 4), (8, 8, 2), (12, 8, 2)])
def test_gradient_ratio_bounds_the_fp32_storage_error_of_gradient_energies(N, lo, hi):
    """Rounding A_l to FP32 moves each entry by at most eps_32/2 of itself, so
    the energy (G^T A G)_vv of a hat-function gradient moves by at most
    eps_32/2 * (|G|^T |A| |G|)_vv, i.e. by at most eps_32/2 * rho_l of itself.
    The FP32 form's choice of level types rests on that bound: it must hold
    for the actual rounding on every level, and on the finest level (rho ~
    alpha / (beta h^2)) the actual worst change comes within a factor 10 of
    it, so rho measures the real loss and not a loose upper bound."""
    p = gen.make_problem("hex", N, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, lo, hi))
    H = oracle.setup(p.A, p.G)
    eps = float(np.finfo(np.float32).eps)
    for l, lv in enumerate(H.levels[:-1]):
        A, G = sp.csr_matrix(lv.A), sp.csr_matrix(lv.G)
        rho = amg.gradient_ratio(A, G)
        den = (G.T @ A @ G).diagonal()
        moved = (G.T @ (A.astype(np.float32).astype(np.float64) - A) @ G).diagonal()
        ok = den > 0
        worst = float(np.max(np.abs(moved[ok]) / den[ok]))
        assert worst <= 0.5 * eps * rho * (1 + 1e-9), (l, worst, rho)
        if l == 0:
            assert worst >= 0.05 * eps * rho, (worst, rho)
            assert rho > 1e6


@pytest.mark.parametrize("N,lo,hi", [(8, 2, 4), (10, 8, 2)])
def test_flexible_cg_equals_cg_for_a_fixed_symmetric_preconditioner(N, lo, hi):
    """The FP32 form runs CG with the Polak-Ribiere beta (r_k - r_{k-1})^T z_k
    / r_{k-1}^T z_{k-1}.  With a fixed SPD preconditioner (the FP64 V-cycle)
    CG keeps r_{k-1}^T z_k = 0, so that beta is the standard one in exact
    arithmetic: the residual histories agree to rounding over the first
    iterations, the iteration counts agree and so do the solutions."""
    p = gen.make_problem("hex", N, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, lo, hi),
                         f=lambda n: fields.rhs_uniform(n, 5))
    H = oracle.setup(p.A, p.G)
    xs, its, hs = oracle.pcg(H, p.A, p.f, flexible=False)
    xf, itf, hf = oracle.pcg(H, p.A, p.f, flexible=True)
    assert its == itf
    hs, hf = np.array(hs[:10]), np.array(hf[:10])
    assert np.abs(hs - hf).max() <= 1e-7 * hs.max()
    assert np.linalg.norm(xs - xf) <= 1e-8 * np.linalg.norm(xs)


def test_flexible_cg_orthogonalises_against_the_last_direction(monkeypatch):
    """With a preconditioner that changes every iteration (here z = D_k r with
    a new random positive diagonal D_k each call) the Polak-Ribiere beta is
    the flexible CG of Notay (2000): it makes each new direction A-orthogonal
    to the previous one, beta_k = -z_k^T A p_{k-1} / p_{k-1}^T A p_{k-1}
    (substitute r_k - r_{k-1} = -alpha A p_{k-1}).  The iterates of the
    oracle's CG must equal those of that explicit form, written out here;
    the standard beta (which assumes r_{k-1}^T z_k = 0) must not."""
    p = gen.make_problem("hex", 4, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 2, 3),
                         f=lambda n: fields.rhs_uniform(n, 9))
    H = oracle.setup(p.A, p.G)
    A = sp.csr_matrix(p.A)
    n = A.shape[0]
    K = 8
    rng = np.random.default_rng(4)
    D = [np.exp(rng.uniform(-1.5, 1.5, n)) for _ in range(K + 2)]
    calls = {"k": 0}

    def varying(H_, r, dtype=np.float64, level=0):
        z = D[calls["k"]] * np.asarray(r, dtype=np.float64)
        calls["k"] += 1
        return z

    x = np.zeros(n)
    r = p.f.copy()
    z = D[0] * r
    d = z.copy()
    for k in range(K):
        q = A @ d
        a = (r @ z) / (d @ q)
        x = x + a * d
        r = r - a * q
        z = D[k + 1] * r
        d = z - ((z @ q) / (d @ q)) * d
    monkeypatch.setattr(amg, "vcycle", varying)
    xf, itf, _ = amg.pcg(H, A, p.f, rtol=1e-30, maxit=K, flexible=True)
    calls["k"] = 0
    xs, its, _ = amg.pcg(H, A, p.f, rtol=1e-30, maxit=K, flexible=False)
    assert itf == its == K
    assert np.linalg.norm(xf - x) <= 1e-10 * np.linalg.norm(x)
    assert np.linalg.norm(xs - x) > 1e-3 * np.linalg.norm(x)


# ----------------------------------------------------------------------------
# the 3D extension reading (case 2 of the block construction) against the
# exact interior harmonic extension: measured, not a pin of the paper
# ----------------------------------------------------------------------------
def _two_grid_factor(H, P, A):
    n = A.shape[0]
    mats = amg._cast(H, np.float64)
    M = mats[0]
    nc = H.levels[0].smoother.ncolors
    up, down = list(range(nc)), list(range(nc - 1, -1, -1))
    z = np.zeros(n)

    def pre(e):
        x = amg._schwarz(M, e.copy(), z, up)
        x = amg._schwarz(M, x, z, down)
        return x - (M["A"] @ x) / M["l1"]

    def post(e):
        x = e - (M["A"] @ e) / M["l1"]
        x = amg._schwarz(M, x, z, up)
        return amg._schwarz(M, x, z, down)
    Ad = A.toarray()
    Epre = np.stack([pre(c) for c in np.eye(n)], axis=1)
    Epost = np.stack([post(c) for c in np.eye(n)], axis=1)
    Pi = P @ np.linalg.solve(P.T @ Ad @ P, P.T @ Ad)
    return float(max(abs(np.linalg.eigvals(Epost @ (np.eye(n) - Pi) @ Epre))))


@pytest.mark.parametrize("alpha", ["iso", "jump"])
def test_depth_ordered_extension_against_exact_interior_extension(alpha):
    """Hex 6^3: the two-grid factor with the depth-ordered block extension
    (the 3D reading) against the exact P_app = R^T - S_I A_II^{-1} S_I^T A R^T
    (eq. (sparseP) with the global A_II^{-1}).  Exact: ~0.07; depth-ordered:
    0.20 (isotropic) and 0.25 (jumps), i.e. the 3D localisation, not the
    smoother, is what limits the method here."""
    al = 1.0 if alpha == "iso" else (lambda m: fields.subdomain_log_uniform(m, 2, 5))
    p = gen.make_problem("hex", 6, beta=1.0, alpha=al)
    H = oracle.setup(p.A, p.G, max_levels=2)
    lv = H.levels[0]
    assert not lv.exact_blocks
    n = p.A.shape[0]
    Rt = amg.r_transpose(lv.rr, n).toarray()
    Ad = p.A.toarray()
    I = lv.interior
    Pex = Rt.copy()
    Pex[I] = Rt[I] - np.linalg.solve(Ad[np.ix_(I, I)], Ad[I] @ Rt)
    r9 = _two_grid_factor(H, lv.P.toarray(), p.A)
    ex = _two_grid_factor(H, Pex, p.A)
    print(f"two-grid factor: depth-ordered {r9:.3f}, exact P_app {ex:.3f}")
    assert ex < 0.1
    assert 0.15 < r9 < 0.3 and r9 > 2.5 * ex


# ----------------------------------------------------------------------------
# patch extension (per-column local harmonic extension, the 3D variant)
# ----------------------------------------------------------------------------
def test_patch_extension_equals_dense_ideal_formula_in_2d():
    """2D: A_II is block diagonal (components of at most 64 DoFs), and
    64 hops from a column's exterior DoFs reach the whole components coupled
    to it (interior DoFs are coupled only inside their component), so the
    per-column patch extension is eq. (sparseP) exactly (dense formula)."""
    for alpha in (1.0, lambda m: fields.stripes_2d(m)):
        p = gen.make_problem("tri", 3, beta=0.01, alpha=alpha)
        H = oracle.setup(p.A, p.G, max_levels=2, ext_mode="patch", patch_hops=64,
                         patch_cap=10 ** 6)
        lv = H.levels[0]
        assert lv.exact_blocks
        n = p.A.shape[0]
        Rt = amg.r_transpose(lv.rr, n).toarray()
        Ad = p.A.toarray()
        I = lv.interior
        Pd = Rt.copy()
        Pd[I] = Rt[I] - np.linalg.solve(Ad[np.ix_(I, I)], Ad[I] @ Rt)
        assert np.abs(lv.P.toarray() - Pd).max() <= 1e-10 * np.abs(Pd).max()


@pytest.mark.parametrize("cap", [16, 128])
def test_patch_columns_are_harmonic_on_their_patch(cap):
    """Every column x = P e_c of the patch form is A-harmonic on its patch,
    (A x)_S = 0, has its exterior values R^T e_c, and is zero on the other
    interior DoFs; the patch is interior, at most `cap` DoFs, and (one hop,
    no cap) exactly the interior DoFs coupled in A to the exterior ones."""
    p = gen.make_problem("hex", 6, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 3, 5))
    H = oracle.setup(p.A, p.G, max_levels=2, ext_mode="patch", patch_hops=2, patch_cap=cap)
    lv = H.levels[0]
    n = p.A.shape[0]
    Rt = amg.r_transpose(lv.rr, n).tocsc()
    P = lv.P.tocsc()
    A = p.A.tocsr()
    isint = np.zeros(n, dtype=bool)
    isint[lv.interior] = True
    assert len(lv.patches) == Rt.shape[1]
    for c in range(0, Rt.shape[1], 7):
        S = lv.patches[c]
        assert len(S) <= cap and isint[S].all()
        x = P[:, c].toarray().ravel()
        ext = Rt.indices[Rt.indptr[c]:Rt.indptr[c + 1]]
        assert np.array_equal(x[~isint], Rt[:, c].toarray().ravel()[~isint])
        off = np.setdiff1d(np.nonzero(isint)[0], S)
        assert not x[off].any()
        Ax = A @ x
        assert np.abs(Ax[S]).max() <= 1e-12 * (abs(A) @ abs(x))[S].max()
    one = amg.patch_sets(p.A, Rt, lv.interior, hops=1, cap=10 ** 6)
    for c in range(0, Rt.shape[1], 11):
        ext = Rt.indices[Rt.indptr[c]:Rt.indptr[c + 1]]
        nb = np.unique(np.concatenate([A.indices[A.indptr[e]:A.indptr[e + 1]] for e in ext]))
        assert np.array_equal(one[c], nb[isint[nb]])


def test_patch_extension_two_grid_factor_against_exact_extension():
    """Hex 6^3 with jumps: the two-grid factor of the patch form lies between
    the exact P_app's (eq. (sparseP) with the global A_II^{-1}) and the
    depth-ordered block form's: a measurement of the 3D localisation, the
    paper has no 3D construction."""
    al = lambda m: fields.subdomain_log_uniform(m, 2, 5)
    p = gen.make_problem("hex", 6, beta=1.0, alpha=al)
    Hb = oracle.setup(p.A, p.G, max_levels=2)
    Hp = oracle.setup(p.A, p.G, max_levels=2, ext_mode="patch")
    lv = Hb.levels[0]
    n = p.A.shape[0]
    Rt = amg.r_transpose(lv.rr, n).toarray()
    Ad = p.A.toarray()
    I = lv.interior
    Pex = Rt.copy()
    Pex[I] = Rt[I] - np.linalg.solve(Ad[np.ix_(I, I)], Ad[I] @ Rt)
    r9 = _two_grid_factor(Hb, lv.P.toarray(), p.A)
    rp = _two_grid_factor(Hb, Hp.levels[0].P.toarray(), p.A)
    ex = _two_grid_factor(Hb, Pex, p.A)
    print(f"two-grid factor: exact {ex:.3f}, patch {rp:.3f}, depth-ordered blocks {r9:.3f}")
    assert ex <= rp + 1e-9 and rp < r9


# ----------------------------------------------------------------------------
# 3D localisations in their unbounded limits: eq. (sparseP) with the global
# A_II^{-1}, computed densely
# ----------------------------------------------------------------------------
def _dense_ideal(p, lv):
    n = p.A.shape[0]
    Rt = amg.r_transpose(lv.rr, n).toarray()
    Ad = p.A.toarray()
    I = lv.interior
    Pd = Rt.copy()
    Pd[I] = Rt[I] - np.linalg.solve(Ad[np.ix_(I, I)], Ad[I] @ Rt)
    return Pd


@pytest.mark.parametrize("N", [6, 8])
def test_block_extension_is_exact_in_3d_when_the_block_bound_admits_components(N):
    """3D: graph(A_II) is one connected component; with a block bound above
    |I| that component is the one block and P is eq. (sparseP) exactly, the
    dense formula with the global A_II^{-1}."""
    p = gen.make_problem("hex", N, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 2, 5))
    H = oracle.setup(p.A, p.G, max_levels=2, ext_block_max=10 ** 6)
    lv = H.levels[0]
    assert lv.exact_blocks and len(lv.blocks) == 1
    Pd = _dense_ideal(p, lv)
    assert np.abs(lv.P.toarray() - Pd).max() <= 1e-10 * np.abs(Pd).max()


def test_patch_extension_is_exact_in_3d_without_cap_and_with_enough_hops():
    """3D, hex 6^3 with jumps: with no cap and one hop more than the diameter
    of graph(A_II) (measured here by BFS), every patch is the whole interior
    set (graph(A_II) is connected), and the per-column least-energy extension
    is column c of eq. (sparseP) with the global A_II^{-1}."""
    p = gen.make_problem("hex", 6, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 2, 5))
    H0 = oracle.setup(p.A, p.G, max_levels=2)
    I = H0.levels[0].interior
    AII = abs(p.A.tocsr()[I][:, I]) > 0
    diam = shortest_path(AII, unweighted=True, directed=False).max()
    assert np.isfinite(diam)
    H = oracle.setup(p.A, p.G, max_levels=2, ext_mode="patch", patch_hops=int(diam) + 1,
                     patch_cap=10 ** 6)
    lv = H.levels[0]
    assert all(np.array_equal(S, np.sort(I)) for S in lv.patches)
    Pd = _dense_ideal(p, lv)
    assert np.abs(lv.P.toarray() - Pd).max() <= 1e-10 * np.abs(Pd).max()


@pytest.mark.parametrize("alpha", ["iso", "jump"])
def test_depth_ordered_blocks_are_harmonic_given_the_shallower_rows(alpha):
    """The 3D block form (bound 64, so A_II is split): for every block B of
    depth d, P restricted to the exterior rows, the rows of blocks of depth
    below d and B's own rows is A-harmonic on B; the couplings of B to the
    other blocks of depth >= d are exactly what the localisation drops.
    Blocks partition the interior set, depths are nondecreasing along the
    processing order and P keeps R^T on the exterior."""
    al = 1.0 if alpha == "iso" else (lambda m: fields.subdomain_log_uniform(m, 2, 5))
    p = gen.make_problem("hex", 6, beta=1.0, alpha=al)
    H = oracle.setup(p.A, p.G, max_levels=2)
    lv = H.levels[0]
    assert not lv.exact_blocks
    n = p.A.shape[0]
    allb = np.concatenate(lv.blocks)
    assert np.array_equal(np.sort(allb), np.sort(lv.interior))
    Pd = lv.P.toarray()
    Ad = p.A.toarray()
    Rt = amg.r_transpose(lv.rr, n).toarray()
    ext = np.setdiff1d(np.arange(n), lv.interior)
    assert np.array_equal(Pd[ext], Rt[ext])
    depths = np.asarray(lv.depths)
    for b, B in enumerate(lv.blocks):
        keep = np.concatenate([ext] + [lv.blocks[k] for k in range(len(lv.blocks))
                                       if depths[k] < depths[b]] + [B])
        res = Ad[np.ix_(B, keep)] @ Pd[keep]
        scale = (abs(Ad[np.ix_(B, keep)]) @ abs(Pd[keep])).max()
        assert np.abs(res).max() <= 1e-12 * max(scale, 1e-300)
    assert len(set(depths.tolist())) > 1
