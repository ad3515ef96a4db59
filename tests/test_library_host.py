"""Host-side checks of the compiled library (no GPU needed): it loads, it
exports every function include/amg.h declares, and its integer setup of the
finest level is bit-exact with the oracle (Algorithms 1-3, G_c, extension
blocks, smoother stars and colours)."""
import os
import re

import numpy as np
import pytest

import gen
from gen import fields
import paper_2602_23613_amd as amglib
from paper_2602_23613_amd import _lib
from oracle import amg
from refsel import RefSelector

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_function():
    lib = _lib.load()
    hdr = open(os.path.join(ROOT, "include", "amg.h")).read()
    names = set(re.findall(r"\b(amg_[a-z0-9_]+)\s*\(", hdr))
    assert names, "no declarations found"
    for nm in sorted(names):
        assert hasattr(lib, nm), nm
    assert set(_lib.EXPORTED) <= names


def oracle_level0(p, ref=None):
    lv = amg.Level(A=p.A, G=p.G)
    lv.Gt, lv.B = amg.augment_g(p.G)
    lv.S = amg.nodal_graph(p.A, lv.Gt)
    if ref is not None:
        cg, bc = ref
        lv.cG, lv.cf = np.sort(cg), None
        Cp = np.concatenate([lv.cG, bc])
    else:
        lv.cG, lv.cf = amg.nodal_cf(lv.S, lv.B)
        Cp = np.concatenate([lv.cG, lv.B])
    n = p.A.shape[0]
    lv.rr, lv.interior = amg.form_r(lv.Gt, Cp, lv.B, n, skip_bb=ref is None)
    lv.blocks, lv.depths, lv.exact_blocks = amg.extension_blocks(
        p.A, lv.Gt, lv.interior, np.concatenate([Cp, lv.rr.k]))
    Gc, cols = amg.coarse_gradient(p.G, lv.rr)
    lv.smoother = amg.smoother_setup(p.A, p.G)
    return lv, Gc, cols


def compare_integers(d, lv, Gc, cols):
    """Assert the library's exported integers equal the oracle level's."""
    if lv.cf is not None:
        assert np.array_equal(d["cf"], lv.cf)
    assert np.array_equal(d["cg"], lv.cG)
    for f in ("dof1", "dof2", "i", "j", "k", "s1", "s2"):
        assert np.array_equal(d["r_" + f], getattr(lv.rr, f)), f
    assert np.array_equal(d["interior"], lv.interior)
    ob = np.concatenate([[0], np.cumsum([len(b) for b in lv.blocks])]).astype(np.int64)
    assert np.array_equal(d["block_ptr"], ob)
    if len(lv.blocks):
        assert np.array_equal(d["block_dofs"], np.concatenate(lv.blocks))
    assert np.array_equal(d["block_depth"], lv.depths)
    assert d["exact_blocks"] == lv.exact_blocks
    sm = lv.smoother
    sp_ = np.concatenate([[0], np.cumsum([len(b) for b in sm.blocks])]).astype(np.int64)
    assert np.array_equal(d["star_ptr"], sp_)
    assert np.array_equal(d["star_dofs"], np.concatenate(sm.blocks))
    assert np.array_equal(d["star_color"], sm.color)
    assert d["ncolors"] == sm.ncolors
    assert np.array_equal(d["gc_ptr"], Gc.indptr)
    assert np.array_equal(d["gc_col"], Gc.indices)
    assert np.array_equal(d["gc_val"], Gc.data.astype(np.int64))
    assert np.array_equal(d["gc_cols"], cols)


CASES = [("tri", 4, {}, 1.0), ("tri", 5, {}, "stripes"), ("hex", 6, {}, 1.0),
         ("hex", 9, {}, "jump"), ("tet", 4, dict(jitter=0.2, mesh_seed=4), "checker"),
         ("tet", 5, dict(jitter=0.2, mesh_seed=7), 1.0)]


def alpha_of(name):
    return {1.0: 1.0, "stripes": lambda m: fields.stripes_2d(m),
            "jump": lambda m: fields.subdomain_log_uniform(m, 3, 2),
            "checker": lambda m: fields.checkerboard(m, 2)}[name]


@pytest.mark.parametrize("kind,size,kw,alpha", CASES)
def test_level0_integers_bit_exact(kind, size, kw, alpha):
    p = gen.make_problem(kind, size, alpha=alpha_of(alpha), **kw)
    d = amglib.level0_integers(p.A, p.G)
    lv, Gc, cols = oracle_level0(p)
    compare_integers(d, lv, Gc, cols)


def test_level0_integers_refinement_mode_bit_exact():
    p = gen.make_problem("tri", 4, beta=0.01)
    lv0 = amg.Level(A=p.A, G=p.G)
    lv0.Gt, lv0.B = amg.augment_g(p.G)
    cg, bc = RefSelector(p)(0, lv0)
    d = amglib.level0_integers(p.A, p.G, interp="ref", ref=[(cg, bc)])
    lv, Gc, cols = oracle_level0(p, ref=(cg, bc))
    compare_integers(d, lv, Gc, cols)


def test_bad_gradient_is_rejected():
    p = gen.make_problem("hex", 3)
    G = p.G.tolil()
    G[0, 5] = 1.0
    G[0, 6] = -1.0   # now three entries in row 0
    with pytest.raises(amglib.AmgError) as e:
        amglib.level0_integers(p.A, G.tocsr())
    assert e.value.status == -4


def test_unsorted_csr_is_rejected():
    p = gen.make_problem("hex", 3)
    A = p.A.copy()
    A.indices[[0, 1]] = A.indices[[1, 0]]
    with pytest.raises(amglib.AmgError) as e:
        amglib.level0_integers(A, p.G)
    assert e.value.status == -3


def test_csr_tuples_are_checked_before_their_pointers_are_passed():
    """A CSR tuple reaches the C ABI as three raw pointers, so the binding
    checks what the library assumes of them: int64 row pointers with
    nrows + 1 entries, int32 column ids, float64 values as many as the
    column ids, contiguous, all host arrays or all CUDA tensors.  Host
    tuples go through the host-only integer setup; every bad variant is
    refused before any library call."""
    p = gen.make_problem("hex", 3)
    A = p.A.tocsr()
    rp = A.indptr.astype(np.int64)
    ci = A.indices.astype(np.int32)
    va = A.data.astype(np.float64)
    n = A.shape[0]
    G = p.G.tocsr()
    Gt = (G.indptr.astype(np.int64), G.indices.astype(np.int32), G.data.astype(np.float64),
          G.shape[0], G.shape[1])
    ref = amglib.level0_integers(A, G)
    got = amglib.level0_integers((rp, ci, va, n, n), Gt)
    assert sorted(ref) == sorted(got)
    assert all(np.array_equal(np.asarray(ref[k]), np.asarray(got[k])) for k in ref)
    bad = [
        ((rp.astype(np.int32), ci, va, n, n), TypeError),
        ((rp, ci.astype(np.int64), va, n, n), TypeError),
        ((rp, ci, va.astype(np.float32), n, n), TypeError),
        ((rp[:-1], ci, va, n, n), ValueError),
        ((rp, ci, va[:-1], n, n), ValueError),
        ((rp, ci, np.repeat(va, 2)[::2], n, n), ValueError),
    ]
    for tup, err in bad:
        with pytest.raises(err):
            amglib.level0_integers(tup, Gt)
    torch = pytest.importorskip("torch")
    cpu = (torch.from_numpy(rp), torch.from_numpy(ci), torch.from_numpy(va), n, n)
    with pytest.raises(TypeError):
        amglib.level0_integers(cpu, Gt)


def test_noalloc_spmv_dot_rejects_sizes_beyond_its_scratch():
    """The allocation-free SpMV-with-dot checks its partial-sum count against
    the static scratch before any HIP call: a 20M-row descriptor (mean row
    length 1: 4 lanes, 64 rows per workgroup, 312,500 partials) is refused
    with AMG_ERR_LIMIT.  Nothing is launched, so host buffers stand in for
    device ones."""
    import ctypes as C
    lib = _lib.load()
    n = 20_000_000
    rp = np.zeros(2, dtype=np.int64)
    ci = np.zeros(1, dtype=np.int32)
    va = np.zeros(1)
    a = _lib.amg_csr()
    a.nrows, a.ncols, a.nnz = n, n, n
    a.rowptr, a.colidx, a.val = rp.ctypes.data, ci.ctypes.data, va.ctypes.data
    a.on_device = 1
    buf = np.zeros(4)
    st = lib.amg_spmv_dot_noalloc(C.byref(a), buf.ctypes.data, buf.ctypes.data,
                                  buf.ctypes.data, None)
    assert st == -9, _lib.STATUS.get(st, st)
    assert b"static scratch" in lib.amg_last_error()


@pytest.mark.parametrize("kind,size,cap", [("hex", 6, 128), ("hex", 6, 16), ("hex", 8, 40), ("tri", 4, 128),
                                           ("tet", 4, 64)])
def test_patch_sets_bit_exact(kind, size, cap):
    """The patch extension's per-column interior supports (integer graph work
    on the host) equal the oracle's patch_sets."""
    kw = dict(jitter=0.2, mesh_seed=4) if kind == "tet" else {}
    p = gen.make_problem(kind, size, beta=1.0, alpha=lambda m: fields.subdomain_log_uniform(m, 2, 7), **kw)
    d = amglib.level0_integers(p.A, p.G, ext_mode="patch", patch_hops=2, patch_cap=cap)
    lv, _, _ = oracle_level0(p)
    n = p.A.shape[0]
    ps = amg.patch_sets(p.A, amg.r_transpose(lv.rr, n), lv.interior, hops=2, cap=cap)
    ptr = np.concatenate([[0], np.cumsum([len(x) for x in ps])]).astype(np.int64)
    assert np.array_equal(d["patch_ptr"], ptr)
    assert np.array_equal(d["patch_dofs"], np.concatenate(ps))
    assert max(len(x) for x in ps) <= cap


def test_patch_options_are_checked():
    """Patch sizes beyond what the kernel's LDS holds, or no hops, are
    refused before any work (AMG_ERR_ARG)."""
    p = gen.make_problem("hex", 4, beta=1.0)
    for bad in (dict(patch_cap=193), dict(patch_cap=0), dict(patch_hops=0), dict(patch_hops=9)):
        with pytest.raises(amglib.AmgError) as e:
            amglib.level0_integers(p.A, p.G, ext_mode="patch", **bad)
        assert e.value.status == -1, bad
